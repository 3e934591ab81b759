"""Four-column solves of several handles on one device share one Krylov
workspace: each handle's batch keeps only its matrices, the workspace grows
to the largest batch's sizes, and solves on the grown workspace (graph
replay included: graphs captured on the old arrays are dropped) give the
same bits as before it grew and match one-column solves."""

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


def _system(n, seed):
    sc = synth.regular_3d(n=n, k_par=1e4, kappa=1e-4, seed=seed)
    fs = [None] + [synth.host_sources(sc, 100 + seed * 10 + k) for k in range(3)]
    A, B, part = tpfa.assemble(sc, sources=fs)
    return sc, fs, A, dev(B.T.copy()), part


def _four(s, bt):
    x = torch.zeros_like(bt)
    rc, st = L.mdp_solve(s.handle, bt, x)
    assert rc == L.MDP_OK
    return x, st


def test_batches_share_one_workspace_that_grows():
    small = _system(10, 1)
    big = _system(16, 2)
    s_small = Solver(small[2], small[4], precision="fp64", flags=L.MDP_GRAPHS)
    s_big = Solver(big[2], big[4], precision="mixed")
    s_mid = Solver(small[2], small[4], precision="mixed")
    base = L.mdp_multi_rhs_memory(s_small.handle)["held"]
    assert base == 0, f"four-column batches of other handles still hold {base} bytes"
    try:
        say("[multi-rhs] small FP64 handle, first batch")
        x1, st1 = _four(s_small, small[3])
        m1 = L.mdp_multi_rhs_memory(s_small.handle)
        assert m1["plan_bytes"] > 0 and m1["shared_bytes"] > 0
        assert m1["held"] == m1["plan_bytes"] + m1["shared_bytes"]
        say("[multi-rhs] big mixed handle: the workspace grows")
        xb, stb = _four(s_big, big[3])
        mb = L.mdp_multi_rhs_memory(s_big.handle)
        assert mb["shared_bytes"] > m1["shared_bytes"]
        assert L.mdp_multi_rhs_memory(s_small.handle)["shared_bytes"] == mb["shared_bytes"]
        assert mb["held"] == m1["plan_bytes"] + mb["plan_bytes"] + mb["shared_bytes"]
        say("[multi-rhs] small handle again on the grown workspace")
        x2, st2 = _four(s_small, small[3])
        assert torch.equal(x1, x2) and [s["iters"] for s in st1] == [s["iters"] for s in st2]
        _four(s_mid, small[3])
        mm = L.mdp_multi_rhs_memory(s_mid.handle)
        assert mm["shared_bytes"] == mb["shared_bytes"]  # fits: no growth
        assert mm["held"] == m1["plan_bytes"] + mb["plan_bytes"] + mm["plan_bytes"] + mb["shared_bytes"]
        for (sc, fs, A, bt, part), s, x, st in ((small, s_small, x2, st2), (big, s_big, xb, stb)):
            for k in range(4):
                xk, stk = s.solve(bt[k].clone())
                assert abs(st[k]["iters"] - stk[0]["iters"]) <= 1
                assert relerr(host(x[k]), host(xk)) <= 1e-6
                Ao, bo, _ = oa.assemble(sc if fs[k] is None else sc.with_source(fs[k]))
                assert np.linalg.norm(bo - Ao @ host(x[k])) <= 1e-8 * np.linalg.norm(bo)
    finally:
        s_big.close()
        held = L.mdp_multi_rhs_memory(s_small.handle)["held"]
        s_mid.close()
        s_small.close()
    say(f"[multi-rhs] held after the big handle went: {held}")
    probe = Solver(small[2], small[4], precision="fp64")
    try:
        assert L.mdp_multi_rhs_memory(probe.handle)["held"] == 0  # the last batch took the workspace along
    finally:
        probe.close()
