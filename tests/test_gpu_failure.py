"""Failure handling of the solve, with each condition forced from the host:
stagnation (a tolerance below what FP64 rounding lets the true residual
reach) and the mixed-to-FP64 fallback (matrix values beyond FP32's range, so
the FP32 preconditioner turns them into Inf/NaN; and mixed-precision
stagnation).  No kernel is made to fault: the non-finite values are ordinary
IEEE arithmetic, caught by the Arnoldi step's own checks."""

import numpy as np
import pytest
import torch

import synth
from oracle import assembly as oa
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu

ANY = (L.MDP_OK, L.MDP_NOT_CONVERGED, L.MDP_STAGNATED, L.MDP_ENAN)
BEYOND_FP32 = 1e40  # FP32's largest finite value is about 3.4e38


@pytest.fixture(scope="module")
def system():
    sc = synth.regular_3d(n=12, k_par=1e4, kappa=1e-4, seed=5)
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    ref, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-13))
    return {"A": A, "b": b, "part": part, "x": ref.x}


def _solve(s, b):
    x = torch.zeros_like(b)
    rc, st = L.mdp_solve(s.handle, b, x, None, ok=ANY)
    return rc, st[0], host(x)


@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_tolerance_below_rounding_floor_stagnates(system, prec):
    """rtol = 1e-18 cannot be met in FP64: the solve stops with
    MDP_STAGNATED well before max_iter, at a residual near rounding level,
    with the oracle's solution."""
    say(f"[failure] stagnation {prec}")
    s = Solver(system["A"], system["part"], precision=prec, rtol=1e-18)
    try:
        rc, st, x = _solve(s, dev(system["b"]))
        say(f"[failure] {prec}: {st}")
        assert rc == L.MDP_STAGNATED and st["status"] == L.MDP_STAGNATED
        assert st["converged"] == 0 and st["fallback"] == 0
        assert st["iters"] < 1000
        assert st["rel_res_true"] <= 1e-12
        assert relerr(x, system["x"]) <= 1e-9
    finally:
        s.close()


def test_stagnation_in_a_batch(system):
    """Each pair of a batch stops on its own stagnation."""
    say("[failure] stagnation in a batch")
    ss = [Solver(system["A"], system["part"], rtol=1e-18) for _ in range(2)]
    try:
        bs = [dev(system["b"]), dev(2.0 * system["b"])]
        xs = [torch.zeros_like(b) for b in bs]
        rc, st = L.mdp_solve_batch([s.handle for s in ss], bs, xs, None)
        assert rc == L.MDP_STAGNATED
        for k in range(2):
            assert st[k]["status"] == L.MDP_STAGNATED and st[k]["iters"] < 1000
            assert relerr(host(xs[k]), (k + 1) * system["x"]) <= 1e-9
    finally:
        for s in ss:
            s.close()


def test_mixed_overflow_reports_nan_without_fallback(system):
    say("[failure] mixed, matrix beyond FP32 range, no fallback")
    s = Solver(system["A"] * BEYOND_FP32, system["part"], precision="mixed")
    try:
        rc, st, _ = _solve(s, dev(system["b"] * BEYOND_FP32))
        assert rc == L.MDP_ENAN and st["status"] == L.MDP_ENAN and st["fallback"] == 0
    finally:
        s.close()


@pytest.mark.parametrize("graphs", [False, True])
def test_mixed_overflow_falls_back_to_fp64(system, graphs):
    """With MDP_FALLBACK_FP64 the column is solved again in FP64: converged,
    the oracle's solution, and iterations = those of the failed mixed attempt
    plus those of a plain FP64 handle.  Two solves in a row on one handle (the
    second replays the FP64 steps' graphs when MDP_GRAPHS is set) agree."""
    A, b = system["A"] * BEYOND_FP32, system["b"] * BEYOND_FP32
    flags = L.MDP_FALLBACK_FP64 | (L.MDP_GRAPHS if graphs else 0)
    say(f"[failure] mixed overflow with fallback, graphs={graphs}")
    s_nan = Solver(A, system["part"], precision="mixed")
    s64 = Solver(A, system["part"], precision="fp64")
    s = Solver(A, system["part"], precision="mixed", flags=flags)
    try:
        _, st_nan, _ = _solve(s_nan, dev(b))
        _, st64, x64 = _solve(s64, dev(b))
        xs = []
        for k in range(2):
            rc, st, x = _solve(s, dev(b))
            say(f"[failure] solve {k}: {st}")
            assert rc == L.MDP_OK and st["converged"] == 1 and st["fallback"] == 1
            assert st["iters"] == st_nan["iters"] + st64["iters"]
            assert st["restarts"] == st_nan["restarts"] + st64["restarts"] + 1
            assert relerr(x, system["x"]) <= 1e-6 and relerr(x, x64) <= 1e-12
            xs.append(x)
        assert relerr(xs[1], xs[0]) <= 1e-14
    finally:
        for t in (s_nan, s64, s):
            t.close()


def test_mixed_stagnation_falls_back_and_reports_the_second_attempt(system):
    say("[failure] mixed stagnation with fallback")
    s = Solver(system["A"], system["part"], precision="mixed", rtol=1e-18, flags=L.MDP_FALLBACK_FP64)
    s_m = Solver(system["A"], system["part"], precision="mixed", rtol=1e-18)
    try:
        _, st_m, _ = _solve(s_m, dev(system["b"]))
        rc, st, x = _solve(s, dev(system["b"]))
        say(f"[failure] {st}")
        assert rc == L.MDP_STAGNATED and st["fallback"] == 1
        assert st["iters"] > st_m["iters"]
        assert relerr(x, system["x"]) <= 1e-9
    finally:
        s.close()
        s_m.close()


def test_fallback_flag_is_inert_when_nothing_fails(system):
    say("[failure] fallback flag on ordinary solves")
    for prec in ("fp64", "mixed"):
        s0 = Solver(system["A"], system["part"], precision=prec)
        s1 = Solver(system["A"], system["part"], precision=prec, flags=L.MDP_FALLBACK_FP64)
        try:
            _, st0, x0 = _solve(s0, dev(system["b"]))
            _, st1, x1 = _solve(s1, dev(system["b"]))
            assert st1["fallback"] == 0 and st1["iters"] == st0["iters"] and st1["status"] == L.MDP_OK
            assert np.array_equal(x0, x1)
        finally:
            s0.close()
            s1.close()


def test_four_column_group_falls_back_column_by_column(system):
    """mdp_solve with four columns runs them as one group; with matrix values
    beyond FP32's range every column fails in mixed precision and is solved
    again in FP64: converged, fallback = 1, the oracle's solution (scaled
    right-hand sides give scaled solutions)."""
    A, b = system["A"] * BEYOND_FP32, system["b"] * BEYOND_FP32
    say("[failure] four-column group with fallback")
    s = Solver(A, system["part"], precision="mixed", flags=L.MDP_FALLBACK_FP64)
    try:
        B = dev(np.stack([b * (k + 1) for k in range(4)]))
        X = torch.zeros_like(B)
        rc, st = L.mdp_solve(s.handle, B, X, None, ok=ANY)
        say(f"[failure] group stats {[(c['status'], c['iters'], c['fallback']) for c in st]}")
        assert rc == L.MDP_OK
        assert L.mdp_multi_rhs_memory(s.handle)["plan_bytes"] > 0  # the four columns ran as one group
        for k in range(4):
            assert st[k]["converged"] == 1 and st[k]["fallback"] == 1
            assert relerr(host(X[k]), (k + 1) * system["x"]) <= 1e-6
    finally:
        s.close()


def test_batch_pairs_fall_back_one_by_one(system):
    """mdp_solve_batch in mixed precision on matrices beyond FP32's range:
    every pair fails in the batch and, with MDP_FALLBACK_FP64 on its handle,
    is solved again in FP64; a handle without the flag keeps MDP_ENAN."""
    A, b = system["A"] * BEYOND_FP32, system["b"] * BEYOND_FP32
    say("[failure] batch pairs with fallback")
    ss = [Solver(A, system["part"], precision="mixed", flags=L.MDP_FALLBACK_FP64) for _ in range(2)]
    plain = Solver(A, system["part"], precision="mixed")
    try:
        bs = [dev(b), dev(2.0 * b), dev(b)]
        xs = [torch.zeros_like(t) for t in bs]
        rc, st = L.mdp_solve_batch([ss[0].handle, ss[1].handle, plain.handle], bs, xs, None, ok=ANY)
        say(f"[failure] batch stats {[(c['status'], c['iters'], c['fallback']) for c in st]}")
        assert rc == L.MDP_ENAN
        for k in range(2):
            assert st[k]["converged"] == 1 and st[k]["fallback"] == 1 and st[k]["status"] == L.MDP_OK
            assert relerr(host(xs[k]), (k + 1) * system["x"]) <= 1e-6
        assert st[2]["status"] == L.MDP_ENAN and st[2]["fallback"] == 0
    finally:
        for s in ss + [plain]:
            s.close()
