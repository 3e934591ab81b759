"""Batches whose systems all have four right-hand sides (Section 5's
multiple-right-hand-side setting): the preconditioner's matrices are stored
once and every sparse product applies them to the four right-hand sides in
one pass.  Each pair must meet the oracle's residual check and match the same
system solved alone (iterations within one, solution within 1e-6), for the
three block forms, two V-cycles, dense and swept coarsest levels, systems
without fractures, and batches split into chunks."""

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

NRHS = 4
FORMS = {"lower": L.MDP_BLOCK_LOWER, "diag": L.MDP_BLOCK_DIAG, "upper": L.MDP_BLOCK_UPPER}


def _cases():
    """(scenario, set-up options): several AMG levels, a swept coarsest level,
    dense coarsest levels of different sizes, a 3D system, no fractures."""
    return [
        (synth.random_2d(0, n_range=(24, 90), max_segments=8), {}),
        (synth.random_2d(1, n_range=(24, 90), max_segments=8), dict(max_coarse=50)),
        (synth.random_2d(2, n_range=(24, 90), max_segments=8), dict(max_dense=10, max_levels=2)),
        (synth.regular_3d(n=12, k_par=1e4, kappa=1e-4, seed=4), dict(max_coarse=50)),
        (synth.Scenario(2, 20, np.ones(400), [], {(0, 0): 1.0, (0, 1): 0.0}), {}),  # no fractures
        (synth.random_2d(3, n_range=(24, 90), max_segments=8), {}),
    ]


def _build(prec, form="lower", cycles=1, cases=None):
    solvers, bs, srcs, scs = [], [], [], []
    for i, (sc, kw) in enumerate(cases or _cases()):
        fs = [synth.host_sources(sc, 100 * i + k) for k in range(NRHS)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        solvers.append(Solver(A, part, precision=prec, block_form=FORMS[form], vcycles=cycles, **kw))
        bs.append(dev(B.T.copy()))
        srcs.append(fs)
        scs.append(sc)
    return solvers, bs, srcs, scs


def _check_against_single(solvers, bs, srcs, scs, xs, st, need_converged=True):
    k = 0
    for i, sc in enumerate(scs):
        for r in range(NRHS):
            xb = host(xs[i][r])
            x1, st1 = solvers[i].solve(dev(bs[i][r].cpu().numpy()))
            d = relerr(xb, host(x1))
            Ao, bo, _ = oa.assemble(sc.with_source(srcs[i][r]))
            res = np.linalg.norm(bo - Ao @ xb) / np.linalg.norm(bo)
            say(f"    sys={i} rhs={r} n={Ao.shape[0]} iters batch={st[k]['iters']} alone={st1[0]['iters']} "
                f"res={res:.2e} diff={d:.2e}")
            assert st[k]["converged"] == st1[0]["converged"]
            if need_converged or st1[0]["converged"]:
                assert st[k]["converged"] == 1 and res <= 1e-8
                assert abs(st[k]["iters"] - st1[0]["iters"]) <= 1
                assert d <= 1e-6
            k += 1


@pytest.mark.parametrize("prec,form,cycles", [
    ("mixed", "lower", 1), ("fp64", "lower", 1), ("mixed", "upper", 1), ("fp64", "upper", 1),
    ("mixed", "diag", 1), ("mixed", "lower", 2)])
def test_four_rhs_batch_matches_single_solves(prec, form, cycles, capfd, monkeypatch):
    monkeypatch.setenv("MDP_SETUP_VERBOSE", "1")
    solvers, bs, srcs, scs = _build(prec, form, cycles)
    say(f"[batch-rhs] prec={prec} form={form} cycles={cycles} systems={len(scs)} pairs={NRHS * len(scs)}")
    try:
        xs = [torch.zeros_like(b) for b in bs]
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        err = capfd.readouterr().err
        assert f"{NRHS} right-hand-side blocks of {len(scs)} systems" in err  # shared matrices in use
        assert rc == L.MDP_OK or form == "diag"
        _check_against_single(solvers, bs, srcs, scs, xs, st, need_converged=form != "diag")
        # a second call with the cached plan gives the same bits
        xs2 = [torch.zeros_like(b) for b in bs]
        L.mdp_solve_batch([s.handle for s in solvers], bs, xs2)
        for a, b in zip(xs, xs2):
            assert torch.equal(a, b)
    finally:
        for s in solvers:
            s.close()


def test_four_rhs_single_system():
    """One system with four right-hand sides: no row maps, the pair of a
    block's rows is the block itself."""
    sc = synth.regular_3d(n=10, k_par=1e4, kappa=1e4, seed=7)
    solvers, bs, srcs, scs = _build("mixed", cases=[(sc, dict(max_coarse=50))])
    say("[batch-rhs] one system, four right-hand sides")
    try:
        xs = [torch.zeros_like(b) for b in bs]
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        assert rc == L.MDP_OK
        _check_against_single(solvers, bs, srcs, scs, xs, st)
    finally:
        for s in solvers:
            s.close()


def test_four_rhs_with_zero_and_repeated_rhs():
    """Right-hand sides that stop at different times inside one block: a zero
    right-hand side (no iteration), two equal ones, and a distinct one."""
    sc = synth.random_2d(11, n_range=(40, 70), max_segments=8)
    f = synth.host_sources(sc, 5)
    fs = [f, f, synth.host_sources(sc, 6), np.zeros_like(f)]
    A, B, part = tpfa.assemble(sc, sources=fs)
    s = Solver(A, part, precision="mixed", max_coarse=50)
    try:
        bt = dev(B.T.copy())
        bt[3].zero_()
        x = torch.zeros_like(bt)
        say("[batch-rhs] zero and repeated right-hand sides")
        rc, st = L.mdp_solve_batch([s.handle], [bt], [x])
        assert rc == L.MDP_OK
        assert st[3]["iters"] == 0 and torch.count_nonzero(x[3]).item() == 0
        assert torch.equal(x[0], x[1])
        for r in range(3):
            x1, st1 = s.solve(bt[r].clone())
            assert abs(st[r]["iters"] - st1[0]["iters"]) <= 1
            assert relerr(host(x[r]), host(x1)) <= 1e-6
    finally:
        s.close()


def test_four_rhs_chunks(monkeypatch, capfd):
    """Chunks are cut between systems, so each chunk keeps its systems' four
    right-hand sides together; the results agree with the one-chunk batch."""
    monkeypatch.setenv("MDP_SETUP_VERBOSE", "1")
    solvers, bs, srcs, scs = _build("mixed")
    hs = [s.handle for s in solvers]
    try:
        one = [torch.zeros_like(b) for b in bs]
        rc, st1 = L.mdp_solve_batch(hs, bs, one)
        assert rc == L.MDP_OK
        nmax = max(s.n for s in solvers)
        capfd.readouterr()
        monkeypatch.setenv("MDP_BATCH_MAX_UNKNOWNS", str(2 * NRHS * nmax))
        xs = [torch.zeros_like(b) for b in bs]
        rc, st = L.mdp_solve_batch(hs, bs, xs)
        err = capfd.readouterr().err
        lines = [ln for ln in err.splitlines() if "[mdp] batch:" in ln]
        say(f"[batch-rhs] chunks: {lines}")
        assert len(lines) >= 2 and all(f"{NRHS} right-hand-side blocks" in ln for ln in lines)
        assert rc == L.MDP_OK
        for a, b in zip(st, st1):
            assert a["converged"] == 1 and abs(a["iters"] - b["iters"]) <= 1
        for a, b in zip(xs, one):
            assert relerr(host(a), host(b)) <= 1e-6
    finally:
        for s in solvers:
            s.close()


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_four_rhs_initial_guesses_and_budget(prec):
    """Shared matrices with MDP_USE_X0 (each pair starts from its own guess,
    gathered in the internal right-hand-side-major order) and with an
    iteration budget that stops some pairs unconverged: every pair matches
    its solve alone, stats land in the caller's order."""
    cases = [(synth.random_2d(21, n_range=(40, 70), max_segments=6), dict(max_coarse=50)),
             (synth.regular_3d(n=10, k_par=1e4, kappa=1e-4, seed=6), dict(max_coarse=50))]
    for flags, max_iter in ((L.MDP_USE_X0, 1000), (0, 6)):
        solvers, bs, x0s = [], [], []
        for i, (sc, kw) in enumerate(cases):
            fs = [synth.host_sources(sc, 300 + 10 * i + k) for k in range(NRHS)]
            A, B, part = tpfa.assemble(sc, sources=fs)
            solvers.append(Solver(A, part, precision=prec, flags=flags, max_iter=max_iter, **kw))
            bs.append(dev(B.T.copy()))
            x0s.append(dev(np.stack([synth.random_vector(A.shape[0], 700 + 10 * i + k) * 0.1 for k in range(NRHS)])))
        say(f"[batch-rhs] prec={prec} flags={flags} max_iter={max_iter}")
        try:
            xs = [x0.clone() for x0 in x0s]
            rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
            k = 0
            for i, s in enumerate(solvers):
                for r in range(NRHS):
                    x1 = x0s[i][r].clone()
                    _, st1 = s.solve(bs[i][r].clone(), x1)
                    assert st[k]["converged"] == st1[0]["converged"]
                    assert abs(st[k]["iters"] - st1[0]["iters"]) <= 1
                    if max_iter < 1000:
                        assert st[k]["iters"] <= max_iter
                    d = relerr(host(xs[i][r]), host(x1))
                    say(f"    sys={i} rhs={r} iters={st[k]['iters']}/{st1[0]['iters']} conv={st[k]['converged']} diff={d:.1e}")
                    assert d <= (1e-6 if st1[0]["converged"] else 1e-3)
                    k += 1
            if max_iter < 1000:
                assert rc == L.MDP_NOT_CONVERGED
        finally:
            for s in solvers:
                s.close()
