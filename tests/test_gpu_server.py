"""Serving (mdp_server_*): requests on several resident systems run
concurrently in slots with continuous admission.  Each request's result must
be bit-identical to the same solve made alone with mdp_solve, whatever else
is in flight and whether or not its workspace was freed and re-created in
between; a memory budget smaller than one workspace still completes every
request (one at a time).  Poll semantics: PENDING until done, then the final
code once; a collected ticket is unknown."""

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
        fs = [None] + [synth.host_sources(sc, 100 * i + k) for k in (1, 2)]
        A, B, part = tpfa.assemble(sc, sources=fs)
        prec = "mixed" if (prec_mix and i % 2) else "fp64"
        solvers.append(Solver(A, part, precision=prec))
        # one single-rhs request per column, and one request holding all columns
        for k in range(B.shape[1]):
            reqs.append((i, dev(B[:, k].copy()), (sc, fs[k])))
        reqs.append((i, dev(B.T.copy()), None))
    return solvers, reqs


def _alone(solvers, reqs):
    out = []
    for i, b, _ in reqs:
        x = torch.zeros_like(b)
        rc, st = L.mdp_solve(solvers[i].handle, b, x)
        assert rc == L.MDP_OK
        out.append((x, st))
    torch.cuda.synchronize()
    return out


def _serve(solvers, reqs, budget, slots, order):
    srv = L.mdp_server_create(budget, slots)
    try:
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
    xs, res, saw_pending = _serve(solvers, reqs, budget, slots, order)
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
