"""Edge cases of the GPU path against the oracle (dense LAPACK solutions of
the oracle's own assembly): the smallest systems (one host cell; one
fracture cell), sizes on and just past 1024 unknowns, systems whose Arnoldi
tiles have the largest length (true residual of the oracle's matrix), an empty
batch and systems with no right-hand side in a batch, a batch mixing a zero
right-hand side with others, and an exhausted iteration budget."""

import numpy as np
import pytest
import torch

import synth
from synth import Fracture, Scenario
from oracle import assembly as oa
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu

DIR = {(0, 0): 1.0, (0, 1): 0.0}


def _tiny_cases():
    return {
        "one-host-cell": Scenario(2, 1, np.ones(1), [], DIR),
        "one-fracture-cell": Scenario(2, 2, np.ones(4), [Fracture(0, 1, (0,), (1,), 10.0, 0.5, 1e-2)], DIR),
        "tile-1024": Scenario(2, 32, np.ones(1024), [], DIR),
        "tile-1024-plus-1": Scenario(2, 32, np.ones(1024), [Fracture(1, 9, (4,), (5,), 3.0, 2.0, 1e-3)], DIR),
        "3d-one-cell": Scenario(3, 1, np.ones(1), [], DIR),
    }


@pytest.mark.parametrize("name", list(_tiny_cases()))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_smallest_and_tile_boundary_systems(name, prec):
    sc = _tiny_cases()[name]
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    x_ref = osv.solve_dense(Ao, bo)
    say(f"[edges] {name} n={A.shape[0]} prec={prec}")
    s = Solver(A, part, precision=prec)
    try:
        x, st = s.solve(dev(b))
        assert st[0]["converged"] == 1
        assert np.linalg.norm(bo - Ao @ host(x)) <= 1e-8 * np.linalg.norm(bo)
        assert relerr(host(x), x_ref) <= 1e-6
    finally:
        s.close()


def _tile_limit_cases():
    """768^2 = 256 x 2304 unknowns: 256 tiles of exactly the largest tile
    length; with a fracture, 512 tiles shared between the Omega and Gamma
    ranges in proportion to their lengths."""
    k = synth.scenarios._lognormal(768 * 768, seed=3, sigma=1.0)
    return {
        "tile-2304x256": Scenario(2, 768, k, [], DIR),
        "tile-2304x256-plus-fracture": Scenario(2, 768, k, [Fracture(1, 300, (100,), (400,), 1e3, 1e-2, 1e-3)], DIR),
    }


@pytest.mark.parametrize("name", list(_tile_limit_cases()))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_largest_tile_systems(name, prec):
    sc = _tile_limit_cases()[name]
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    say(f"[edges] {name} n={A.shape[0]} prec={prec}")
    s = Solver(A, part, precision=prec)
    try:
        x, st = s.solve(dev(b))
        res = np.linalg.norm(bo - Ao @ host(x)) / np.linalg.norm(bo)
        say(f"    iters={st[0]['iters']} res={res:.2e}")
        assert st[0]["converged"] == 1 and res <= 1e-8
    finally:
        s.close()


def test_empty_batches():
    sc = synth.grid_2d_four_lines(16)
    A, b, part = tpfa.assemble(sc)
    s1 = Solver(A, part)
    s2 = Solver(A, part)
    say("[edges] empty batches")
    try:
        rc = L.lib.mdp_solve_batch(None, 0, None, None, None, None, None)
        assert rc == L.MDP_EINVAL  # NULL arrays are refused even when empty
        bt = dev(b)
        empty = torch.empty((0, A.shape[0]), dtype=torch.float64, device="cuda:0")
        rc, st = L.mdp_solve_batch([s1.handle, s2.handle], [empty, empty], [empty.clone(), empty.clone()])
        assert rc == L.MDP_OK and st == []  # nothing to solve
        x = torch.zeros_like(bt)
        rc, st = L.mdp_solve_batch([s1.handle, s2.handle], [empty, bt], [empty.clone(), x])
        assert rc == L.MDP_OK and st[0]["converged"] == 1
        x1, _ = s1.solve(bt)
        assert relerr(host(x), host(x1)) <= 1e-6
    finally:
        s1.close()
        s2.close()


def test_batch_with_zero_right_hand_side():
    scs = [synth.grid_2d_four_lines(16), synth.regular_3d(n=10, seed=2)]
    solvers, bs = [], []
    for sc in scs:
        A, b, part = tpfa.assemble(sc)
        solvers.append(Solver(A, part, precision="mixed"))
        bs.append(dev(b))
    bs[0] = torch.zeros_like(bs[0])
    xs = [torch.full_like(b, 7.0) for b in bs]
    say("[edges] batch with a zero rhs")
    try:
        rc, st = L.mdp_solve_batch([s.handle for s in solvers], bs, xs)
        assert rc == L.MDP_OK
        assert st[0]["iters"] == 0 and st[0]["converged"] == 1 and not host(xs[0]).any()
        x1, _ = solvers[1].solve(bs[1])
        assert st[1]["converged"] == 1 and relerr(host(xs[1]), host(x1)) <= 1e-6
    finally:
        for s in solvers:
            s.close()


def test_iteration_budget_exhausted():
    sc = synth.regular_3d(n=12, k_par=1e4, kappa=1e4, seed=1)
    A, b, part = tpfa.assemble(sc)
    say("[edges] max_iter 0 and 3")
    for mi in (0, 3):
        s = Solver(A, part, max_iter=mi)
        try:
            x, st = s.solve(dev(b))
            assert st[0]["converged"] == 0 and st[0]["status"] == L.MDP_NOT_CONVERGED
            assert st[0]["iters"] == mi
            if mi == 0:
                assert not host(x).any()
            else:
                r = np.linalg.norm(b - A @ host(x)) / np.linalg.norm(b)
                assert abs(r - st[0]["rel_res_true"]) <= 1e-12 and r < 1.0
        finally:
            s.close()


@pytest.mark.parametrize("scale", [1e-40, 1e30])
@pytest.mark.parametrize("batched", [False, True])
def test_right_hand_sides_outside_fp32_range_in_mixed_mode(scale, batched):
    """Mixed precision with b scaled far outside what FP32 holds at the
    right-hand side's own size (1e-40: below FP32's normal range; 1e30: the
    preconditioner's products would overflow).  The cycle's residual is
    brought to unit norm before the FP32 cast, so the solve is that of the
    unscaled b times the scale: same iteration count, the oracle's solution
    of the scaled system within 1e-6, residual of the oracle's matrix <= 1e-8."""
    sc = synth.regular_3d(n=10, seed=3, k_par=1e4, kappa=1e-4)
    A, b, part = tpfa.assemble(sc)
    Ao, bo, po = oa.assemble(sc)
    say(f"[edges] mixed scale={scale:g} batched={batched}")
    ref, _, _ = osv.solve(Ao, bo * scale, po, osv.SolveOptions(tol=1e-12))
    s = Solver(A, part, precision="mixed")
    try:
        _, st1 = s.solve(dev(b))
        bt = dev(b * scale)
        if batched:
            s2 = Solver(A, part, precision="mixed")
            xs = [torch.zeros_like(bt), torch.zeros_like(bt)]
            rc, sts = L.mdp_solve_batch([s.handle, s2.handle], [bt, dev(b)], xs, None)
            s2.close()
            x, st = host(xs[0]), sts[0]
            assert sts[1]["iters"] == st1[0]["iters"]
        else:
            xt, sts = s.solve(bt)
            x, st = host(xt), sts[0]
        assert st["converged"] == 1 and st["status"] == L.MDP_OK, st
        assert abs(st["iters"] - st1[0]["iters"]) <= 1, (st, st1)
        assert np.linalg.norm(bo * scale - Ao @ x) <= 1e-8 * np.linalg.norm(bo * scale)
        assert relerr(x, ref.x) <= 1e-6
    finally:
        s.close()
