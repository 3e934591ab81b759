"""Batched solves (mdp_solve_batch): uneven systems with several right-hand
sides in one block-diagonal batch.  Each result must meet the oracle's
residual check and match the same system solved alone (same iteration count
within one, solution within the solve tolerance)."""

import numpy as np
import pytest
import torch

import synth
from oracle import assembly as oa
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu


def _systems():
    out = []
    for seed in range(5):
        out.append(synth.random_2d(seed, n_range=(24, 90), max_segments=8))
    out.append(synth.regular_3d(n=12, k_par=1e4, kappa=1e-4, seed=4))
    out.append(synth.random_3d(5, n_range=(10, 16)))
    out.append(synth.Scenario(2, 20, np.ones(400), [], {(0, 0): 1.0, (0, 1): 0.0}))  # no fractures
    return out


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_batch_matches_single_solves(prec):
    scs = _systems()
    nrhs = [1 + (i % 3) for i in range(len(scs))]
    solvers, bs, xs, srcs, mats = [], [], [], [], []
    for i, sc in enumerate(scs):
        fs = [synth.host_sources(sc, 10 * i + k) if k else None for k in range(nrhs[i])]
        A, B, part = tpfa.assemble(sc, sources=fs)
        solvers.append(Solver(A, part, precision=prec))
        bs.append(dev(B.T.copy()))
        xs.append(torch.zeros_like(bs[-1]))
        srcs.append(fs)
        mats.append(A)
    say(f"[batch] prec={prec} systems={len(scs)} pairs={sum(nrhs)}")
    try:
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        assert rc == L.MDP_OK
        k = 0
        for i, sc in enumerate(scs):
            for r in range(nrhs[i]):
                Ao, bo, po = oa.assemble(sc.with_source(srcs[i][r]))
                xb = host(xs[i][r])
                res = np.linalg.norm(bo - Ao @ xb) / np.linalg.norm(bo)
                x1, st1 = solvers[i].solve(dev(bs[i][r].cpu().numpy()))
                d = relerr(xb, host(x1))
                say(f"    sys={i} rhs={r} n={Ao.shape[0]} iters batch={st[k]['iters']} alone={st1[0]['iters']} "
                    f"res={res:.2e} diff={d:.2e}")
                assert st[k]["converged"] == 1 and res <= 1e-8
                assert abs(st[k]["iters"] - st1[0]["iters"]) <= 1
                assert d <= 1e-6
                k += 1
        # second call with the cached plan gives the same answers
        xs2 = [torch.zeros_like(b) for b in bs]
        rc, st2 = L.mdp_solve_batch([s.handle for s in solvers], bs, xs2)
        for a, b in zip(xs, xs2):
            assert torch.equal(a, b)
    finally:
        for s in solvers:
            s.close()


def test_batch_rejects_mixed_precisions():
    sc = synth.grid_2d_four_lines(16)
    A, b, part = tpfa.assemble(sc)
    s1, s2 = Solver(A, part, precision="fp64"), Solver(A, part, precision="mixed")
    try:
        bt = dev(b)
        with pytest.raises(L.MdpError) as e:
            L.mdp_solve_batch([s1.handle, s2.handle], [bt, bt], [torch.zeros_like(bt), torch.zeros_like(bt)])
        assert e.value.code == L.MDP_EINVAL
    finally:
        s1.close()
        s2.close()


def test_batch_split_into_chunks(monkeypatch, capfd):
    """A batch larger than the chunk bound is solved as several block-diagonal
    chunks, one after another, on one shared workspace sized for the largest;
    every pair still converges and agrees with the one-chunk batch."""
    scs = _systems()
    solvers, bs = [], []
    for i, sc in enumerate(scs):
        fs = [None, synth.host_sources(sc, 500 + i)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        solvers.append(Solver(A, part, precision="mixed"))
        bs.append(dev(B.T.copy()))
    hs = [s.handle for s in solvers]
    try:
        one = [torch.zeros_like(b) for b in bs]
        rc, st1 = L.mdp_solve_batch(hs, bs, one)
        assert rc == L.MDP_OK
        nmax = max(s.n for s in solvers)
        monkeypatch.setenv("MDP_SETUP_VERBOSE", "1")
        # cap = the largest system: its two right-hand sides go to separate
        # chunks; 3x: a few systems per chunk
        for cap in (nmax, 3 * nmax):
            monkeypatch.setenv("MDP_BATCH_MAX_UNKNOWNS", str(cap))
            capfd.readouterr()
            xs = [torch.zeros_like(b) for b in bs]
            rc, st = L.mdp_solve_batch(hs, bs, xs)
            chunks = [ln for ln in capfd.readouterr().err.splitlines() if "[mdp] batch:" in ln]
            say(f"[batch-chunks] cap={cap} chunks={len(chunks)} iters={[s['iters'] for s in st]}")
            assert len(chunks) >= 2
            assert rc == L.MDP_OK
            for a, b in zip(st, st1):
                assert a["converged"] == 1 and a["rel_res_true"] <= 1e-8
                assert abs(a["iters"] - b["iters"]) <= 1
            for a, b in zip(xs, one):
                assert relerr(host(a), host(b)) <= 1e-6
        # a smaller batch afterwards rebuilds the plan
        monkeypatch.delenv("MDP_BATCH_MAX_UNKNOWNS")
        xs = [torch.zeros_like(b) for b in bs[:2]]
        rc, st = L.mdp_solve_batch(hs[:2], bs[:2], xs)
        assert rc == L.MDP_OK
        for a, b in zip(xs, one[:2]):
            assert relerr(host(a), host(b)) <= 1e-6
    finally:
        for s in solvers:
            s.close()


@pytest.mark.timeout(600)
def test_batch_at_uneven_2d_workload_sizes():
    """The uneven 2D batch workload at its own sizes: 16 systems with sides
    drawn from 64..512 and 1..20 fracture segments (log-uniform K_par, kappa
    in [1e-4, 1e4]), four right-hand sides each (Dirichlet data alone and
    with three host source fields), mixed precision, one mdp_solve_batch call
    (the four-block layout that shares the preconditioner's matrices).  Every
    pair: converged, residual of the oracle's own matrix and right-hand side
    at most 1e-8, iterations within 2 of the pair solved alone (one column
    through mdp_solve), and the two solutions within 1e-6."""
    scs = [synth.random_2d(s) for s in range(16)]
    solvers, bs, xs, srcs = [], [], [], []
    for i, sc in enumerate(scs):
        fs = [None] + [synth.host_sources(sc, 4 * i + k) for k in range(1, 4)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        solvers.append(Solver(A, part, precision="mixed"))
        bs.append(dev(np.ascontiguousarray(B.T)))
        xs.append(torch.zeros_like(bs[-1]))
        srcs.append(fs)
    say(f"[batch] workload sizes: sides {[sc.n for sc in scs]}, segments {[len(sc.fractures) for sc in scs]}")
    try:
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        assert rc == L.MDP_OK
        k = 0
        worst = 0.0
        for i, sc in enumerate(scs):
            for r in range(4):
                Ao, bo, po = oa.assemble(sc.with_source(srcs[i][r]))
                xb = host(xs[i][r])
                res = np.linalg.norm(bo - Ao @ xb) / np.linalg.norm(bo)
                x1, st1 = solvers[i].solve(bs[i][r].clone())
                d = relerr(xb, host(x1))
                worst = max(worst, d)
                say(f"    sys={i} n={Ao.shape[0]} rhs={r} iters batch={st[k]['iters']} alone={st1[0]['iters']} "
                    f"res={res:.2e} diff={d:.2e}")
                assert st[k]["converged"] == 1 and res <= 1e-8
                assert abs(st[k]["iters"] - st1[0]["iters"]) <= 2
                assert d <= 1e-6
                k += 1
        say(f"[batch] workload sizes: largest batch-vs-alone difference {worst:.2e}")
    finally:
        for s in solvers:
            s.close()


@pytest.mark.parametrize("rhs", [1, 4])
def test_gauss_seidel_batch_matches_single_solves(rhs):
    """A batch with the multicolour Gauss-Seidel smoother: each system is
    coloured on its own and a colour of a batched level spans all systems;
    every pair matches its solve alone."""
    scs = [synth.random_2d(s, n_range=(24, 70), max_segments=6) for s in range(4)]
    scs.append(synth.regular_3d(n=12, k_par=1e4, kappa=1e-4, seed=4))
    solvers, bs, xs = [], [], []
    for i, sc in enumerate(scs):
        fs = [None] + [synth.host_sources(sc, 30 + 4 * i + k) for k in range(rhs - 1)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        solvers.append(Solver(A, part, precision="mixed", smoother=L.MDP_SMOOTH_GS))
        bs.append(dev(np.ascontiguousarray(B.T)) if rhs > 1 else dev(B[:, 0].copy()))
        xs.append(torch.zeros_like(bs[-1]))
    say(f"[batch] gauss-seidel rhs={rhs}")
    try:
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        assert rc == L.MDP_OK
        k = 0
        for i in range(len(scs)):
            cols = [bs[i]] if rhs == 1 else [bs[i][r] for r in range(rhs)]
            outs = [xs[i]] if rhs == 1 else [xs[i][r] for r in range(rhs)]
            for bcol, xcol in zip(cols, outs):
                x1, st1 = solvers[i].solve(bcol.clone())
                assert st[k]["converged"] == 1 and abs(st[k]["iters"] - st1[0]["iters"]) <= 1
                assert relerr(host(xcol), host(x1)) <= 1e-6
                k += 1
    finally:
        for s in solvers:
            s.close()
