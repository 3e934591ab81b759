"""Serving (mdp_server_*): requests on several resident systems run
concurrently in slots with continuous admission.  Without grouping, each
request's result must be bit-identical to the same columns solved alone with
mdp_solve one at a time, whatever else is in flight and whether or not its
workspace was freed and re-created in between; a memory budget smaller than
one workspace still completes every request (one at a time).  With grouping
(an option), queued requests of one system are solved together, four
columns at a time: every result must match its solve alone within the
solver's tolerance and the oracle's residual check, and the server must
report columns solved four at a time.  Poll semantics: PENDING until done,
then the final code once; a collected ticket is unknown."""

import time

import numpy as np
import pytest
import torch

import synth
from oracle import assembly as oa
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, say

pytestmark = pytest.mark.gpu


def _setup(prec_mix=True):
    scs = [synth.random_2d(s, n_range=(30, 80), max_segments=6) for s in range(3)]
    scs.append(synth.regular_3d(n=14, k_par=1e4, kappa=1e-4, seed=1))
    scs.append(synth.random_3d(2, n_range=(10, 14)))
    solvers, reqs = [], []
    for i, sc in enumerate(scs):
        fs = [None] + [synth.host_sources(sc, 100 * i + k) for k in (1, 2, 3)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        prec = "mixed" if (prec_mix and i % 2) else "fp64"
        solvers.append(Solver(A, part, precision=prec))
        # one single-rhs request per column, and one request holding all columns
        for k in range(B.shape[1]):
            reqs.append((i, dev(B[:, k].copy()), (sc, fs[k])))
        reqs.append((i, dev(B.T.copy()), None))
    return solvers, reqs


def _alone(solvers, reqs):
    """Every request's columns solved one at a time with mdp_solve."""
    out = []
    for i, b, _ in reqs:
        x = torch.zeros_like(b)
        sts = []
        for k in range(b.shape[0] if b.dim() == 2 else 1):
            bk, xk = (b[k], x[k]) if b.dim() == 2 else (b, x)
            rc, st = L.mdp_solve(solvers[i].handle, bk, xk)
            assert rc == L.MDP_OK
            sts += st
        out.append((x, sts))
    torch.cuda.synchronize()
    return out


def _serve(solvers, reqs, budget, slots, order, grouping=False, counts=None):
    srv = L.mdp_server_create(budget, slots)
    try:
        L.mdp_server_set_grouping(srv, grouping)
        for s in solvers:
            L.mdp_server_register(srv, s.handle)
        torch.cuda.synchronize()  # right-hand sides are written before submission
        xs = [None] * len(reqs)
        tickets = {}
        for j in order:
            i, b, _ = reqs[j]
            xs[j] = torch.full_like(b, float("nan"))
            torch.cuda.synchronize()
            tickets[L.mdp_submit(srv, solvers[i].handle, b, xs[j])] = j
        res = [None] * len(reqs)
        deadline = time.time() + 120
        pending = dict(tickets)
        saw_pending = False
        while pending:
            assert time.time() < deadline, f"server requests still pending: {sorted(pending.values())}"
            for t in list(pending):
                rc, st = L.mdp_poll(srv, t)
                if rc == L.MDP_PENDING:
                    saw_pending = True
                    continue
                res[pending.pop(t)] = (rc, st)
            time.sleep(0.0005)
        # a collected ticket is unknown to the server
        t0 = next(iter(tickets))
        assert L.lib.mdp_poll(srv, t0, None) == L.MDP_EINVAL
        if counts is not None:
            counts.update(L.mdp_server_counts(srv))
        return xs, res, saw_pending
    finally:
        L.mdp_server_destroy(srv)


@pytest.mark.parametrize("budget,slots", [(0, 4), (0, 1), (1, 3)])
def test_server_results_identical_to_alone(budget, slots):
    solvers, reqs = _setup()
    say(f"[server] budget={budget} slots={slots} systems={len(solvers)} requests={len(reqs)}")
    alone = _alone(solvers, reqs)
    rng = np.random.default_rng(7)
    order = rng.permutation(len(reqs))
    counts = {}
    xs, res, saw_pending = _serve(solvers, reqs, budget, slots, order, grouping=False, counts=counts)
    assert counts["grouped"] == 0 and counts["columns"] == sum(b.numel() // b.shape[-1] for _, b, _ in reqs)
    for j, (i, b, src) in enumerate(reqs):
        rc, st = res[j]
        xa, sta = alone[j]
        assert rc == L.MDP_OK, (j, rc)
        assert [s["iters"] for s in st] == [s["iters"] for s in sta], j
        assert torch.equal(xs[j], xa), f"request {j} (system {i}) differs from its solve alone"
        if src is not None:  # independent check against the oracle's assembly
            Ao, bo, _ = oa.assemble(src[0].with_source(src[1]))
            xh = host(xs[j])
            assert np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo) <= 1e-8
    say(f"[server] ok; saw a pending poll: {saw_pending}")
    for s in solvers:
        s.close()


@pytest.mark.parametrize("slots", [1, 4])
def test_server_grouping_matches_alone_within_tolerance(slots):
    solvers, reqs = _setup()
    say(f"[server] grouping, slots={slots} systems={len(solvers)} requests={len(reqs)}")
    alone = _alone(solvers, reqs)
    order = np.random.default_rng(11).permutation(len(reqs))
    counts = {}
    xs, res, _ = _serve(solvers, reqs, 0, slots, order, grouping=True, counts=counts)
    say(f"[server] counts {counts}")
    # every system has a request of four columns, which alone fills a group
    assert counts["grouped"] >= 4 * len(solvers)
    assert counts["columns"] == sum(b.numel() // b.shape[-1] for _, b, _ in reqs)
    for j, (i, b, src) in enumerate(reqs):
        rc, st = res[j]
        xa, sta = alone[j]
        assert rc == L.MDP_OK, (j, rc)
        for s1, s0 in zip(st, sta):
            assert s1["converged"] == 1 and abs(s1["iters"] - s0["iters"]) <= 1, (j, s1, s0)
        xg, xr = host(xs[j]).ravel(), host(xa).ravel()
        assert np.linalg.norm(xg - xr) <= 1e-6 * np.linalg.norm(xr), j
        if src is not None:
            Ao, bo, _ = oa.assemble(src[0].with_source(src[1]))
            xh = host(xs[j])
            assert np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo) <= 1e-8
    for s in solvers:
        s.close()


def test_server_argument_errors():
    solvers, reqs = _setup(prec_mix=False)
    srv = L.mdp_server_create(0, 2)
    try:
        i, b, _ = reqs[0]
        x = torch.zeros_like(b)
        with pytest.raises(L.MdpError) as e:  # not registered
            L.mdp_submit(srv, solvers[i].handle, b, x)
        assert e.value.code == L.MDP_EINVAL
        L.mdp_server_register(srv, solvers[i].handle)
        L.mdp_server_register(srv, solvers[i].handle)  # registering twice is harmless
        with pytest.raises(ValueError):
            L.mdp_submit(srv, solvers[i].handle, b[:-1], x[:-1])
        with pytest.raises(ValueError):
            L.mdp_poll(srv, 12345)
        assert L.lib.mdp_poll(srv, 12345, None) == L.MDP_EINVAL
        t = L.mdp_submit(srv, solvers[i].handle, b, x)
        deadline = time.time() + 60
        while True:
            rc, st = L.mdp_poll(srv, t)
            if rc != L.MDP_PENDING:
                break
            assert time.time() < deadline
            time.sleep(0.001)
        assert rc == L.MDP_OK and st[0]["converged"] == 1
    finally:
        L.mdp_server_destroy(srv)
    for s in solvers:
        s.close()


def test_server_destroy_drains_queue():
    solvers, reqs = _setup(prec_mix=False)
    alone = _alone(solvers, reqs)
    srv = L.mdp_server_create(0, 2)
    L.mdp_server_set_grouping(srv, False)
    for s in solvers:
        L.mdp_server_register(srv, s.handle)
    torch.cuda.synchronize()
    xs = []
    for i, b, _ in reqs:
        xs.append(torch.zeros_like(b))
        L.mdp_submit(srv, solvers[i].handle, b, xs[-1])
    L.mdp_server_destroy(srv)  # returns after every queued request ran
    for x, (xa, _) in zip(xs, alone):
        assert torch.equal(x, xa)
    for s in solvers:
        s.close()
