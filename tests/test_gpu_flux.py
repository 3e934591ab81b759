"""GPU parity in the paper's own block reading of eq. (4): Omega = the
pressures of every subdomain (host, fractures, explicit intersection lines
and points), Gamma = the interface fluxes (Section 2.1 eqs. (1)-(3);
oracle/mixed_dim.py).  The system is nonsymmetric (A_GO = -A_OG^T) and
A_GG diagonal, so S~ of eq. (7) is the exact Schur complement and Q_GG the
exact inverse.  The library (vectorised assembly, C++ setup, HIP solve) and
the oracle (loop assembly, Python AMG and FGMRES) run independently: M_L on
a seeded vector; whole solves against the oracle at the same tolerance
(iterations within 2, solution within 1e-6), residual of the oracle's
matrix at most 1e-8, and the error against the oracle's 1e-12 solution
reported."""

import numpy as np
import pytest

import synth
from oracle import mixed_dim as md
from oracle import precond
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa_flux
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu

CASES = {
    "2d-four-lines-32": lambda: synth.grid_2d_four_lines(32),
    "2d-tiny-12": lambda: synth.tiny_2d(12, seed=2),
    "2d-random-s5": lambda: synth.random_2d(5, n_range=(64, 100)),
    "3d-regular-12": lambda: synth.regular_3d(n=12, seed=1),
    "3d-regular-20-lo-hi": lambda: synth.regular_3d(n=20, k_par=1e-4, kappa=1e4, seed=2),
    "3d-regular-20-hi-lo": lambda: synth.regular_3d(n=20, k_par=1e4, kappa=1e-4, seed=3),
    "3d-random-s4": lambda: synth.random_3d(4, n_range=(14, 20)),
    "3d-tiny-9": lambda: synth.tiny_3d(9, seed=4),
}
TOL = {"fp64": 1e-11, "mixed": 3e-5}


@pytest.mark.parametrize("name", list(CASES))
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_flux_reading_matches_oracle(name, prec):
    sc = CASES[name]()
    A, b, part, info = tpfa_flux.assemble_flux(sc)
    Ao, bo, po, io = md.assemble_flux(sc)
    say(f"[flux] {name} {prec}: n={A.shape[0]} cells={info['cells']} intersections={info['intersection']} "
        f"points={info['point']} interfaces={info['interface']}")
    M = precond.ML(Ao, po, cycles=1)
    ref8, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-8), M=M)
    ref, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-12), M=M)
    s = Solver(A, part, precision=prec)
    try:
        assert s.info["levels_omega"] == len(M.H_omega.levels)
        x = synth.random_vector(A.shape[0], 41)
        z = host(s.apply(L.MDP_OP_ML, dev(x)))
        assert relerr(z, M.apply(x)) <= TOL[prec]
        xt, st = s.solve(dev(b))
        xh = host(xt)
        res = np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo)
        err8, err = relerr(xh, ref8.x), relerr(xh, ref.x)
        say(f"    iters {st[0]['iters']} (oracle {ref8.iters}) residual {res:.2e} error vs oracle at 1e-8 "
            f"{err8:.2e}, at 1e-12 {err:.2e}")
        assert st[0]["converged"] == 1 and res <= 1e-8
        assert abs(st[0]["iters"] - ref8.iters) <= 2
        assert err8 <= 1e-6
    finally:
        s.close()


@pytest.mark.timeout(600)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_flux_reading_at_cube_60(prec):
    """A 60^3 cube with nine planes in the flux reading (321,489 unknowns:
    216k host cells, 32k fracture cells, 1.6k line cells, 27 points, 71k
    interface fluxes): solve against the oracle."""
    sc = synth.regular_3d(n=60, k_par=1e4, kappa=1e-4, seed=0)
    A, b, part, info = tpfa_flux.assemble_flux(sc)
    Ao, bo, po, io = md.assemble_flux(sc)
    ref8, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-8))
    s = Solver(A, part, precision=prec)
    try:
        xt, st = s.solve(dev(b))
        xh = host(xt)
        res = np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo)
        err8 = relerr(xh, ref8.x)
        say(f"[flux] 60^3 {prec}: n={A.shape[0]} iters {st[0]['iters']} (oracle {ref8.iters}) residual {res:.2e} "
            f"error vs oracle {err8:.2e}")
        assert st[0]["converged"] == 1 and res <= 1e-8 and abs(st[0]["iters"] - ref8.iters) <= 2
        assert err8 <= 1e-6
    finally:
        s.close()


@pytest.mark.parametrize("name", ["2d-four-lines-32", "3d-regular-12", "3d-random-s4"])
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_dimension_aware_aggregation_matches_oracle(name, prec):
    """mdp_setup_labeled with each unknown's subdomain dimension (Section
    3.3, last paragraph): M_L and the whole solve against the oracle built
    with the same labels."""
    sc = CASES[name]()
    A, b, part, info = tpfa_flux.assemble_flux(sc)
    Ao, bo, po, io = md.assemble_flux(sc)
    M = precond.ML(Ao, po, cycles=1, labels=io["labels"])
    ref8, _, _ = osv.solve(Ao, bo, po, osv.SolveOptions(tol=1e-8), M=M)
    s = Solver(A, part, precision=prec, labels=info["labels"])
    try:
        assert s.info["levels_omega"] == len(M.H_omega.levels)
        x = synth.random_vector(A.shape[0], 43)
        z = host(s.apply(L.MDP_OP_ML, dev(x)))
        assert relerr(z, M.apply(x)) <= TOL[prec]
        xt, st = s.solve(dev(b))
        xh = host(xt)
        res = np.linalg.norm(bo - Ao @ xh) / np.linalg.norm(bo)
        say(f"[flux] labelled {name} {prec}: iters {st[0]['iters']} (oracle {ref8.iters}) residual {res:.2e}")
        assert st[0]["converged"] == 1 and res <= 1e-8 and abs(st[0]["iters"] - ref8.iters) <= 2
        assert relerr(xh, ref8.x) <= 1e-6
    finally:
        s.close()
