"""Parity at the measured sizes, in the configuration the benchmark times.

100^3 (1.09M unknowns; nine full planes, log-normal host, seed 0): the
GPU solves in FP64 and in mixed precision against the oracle's own assembly,
AMG hierarchy and FGMRES on the same system -- solution within 1e-6,
iteration count within 2, true residual of the oracle's matrix at most 1e-8
-- and one application of M_L (Algorithm 1) to a seeded vector, compared
element by element over all 1.09M outputs.

160^3 (4.33M unknowns, the largest single-GPU configuration): the same
checks against the oracle's own assembly, hierarchy and FGMRES on one system,
and mixed against FP64."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import assembly as oa
from oracle import solve as osv
from paper_2206_03203_amd import _lib as L
from paper_2206_03203_amd import tpfa
from paper_2206_03203_amd.solver import Solver

from gpu_common import dev, host, relerr, say

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def cube100():
    sc = synth.regular_3d(n=100, k_par=1e4, kappa=1e-4, seed=0)
    say(f"[fullsize] oracle assembly and setup for {sc.name}")
    Ao, bo, po = oa.assemble(sc)
    M = osv.setup(Ao, po)
    res, _, _ = osv.solve(Ao, bo, po, M=M)
    say(f"[fullsize] oracle solved in {res.iters} iterations, residual {res.rel_res_true:.2e}")
    A, b, part = tpfa.assemble(sc)
    return {"sc": sc, "Ao": sp.csr_matrix(Ao), "bo": bo, "M": M, "res": res, "A": A, "b": b, "part": part}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cube100_solve_matches_oracle(cube100, prec):
    c = cube100
    s = Solver(c["A"], c["part"], precision=prec)
    try:
        x, st = s.solve(dev(c["b"]))
        xh = host(x)
        res = np.linalg.norm(c["bo"] - c["Ao"] @ xh) / np.linalg.norm(c["bo"])
        err = relerr(xh, c["res"].x)
        say(f"[fullsize] {prec}: iters {st[0]['iters']} (oracle {c['res'].iters}), residual {res:.2e}, "
            f"error vs oracle {err:.2e}")
        assert st[0]["converged"] == 1
        assert res <= 1e-8
        assert abs(st[0]["iters"] - c["res"].iters) <= 2
        assert err <= 1e-6
    finally:
        s.close()


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 3e-5)])
def test_cube100_preconditioner_elementwise(cube100, prec, tol):
    c = cube100
    s = Solver(c["A"], c["part"], precision=prec)
    try:
        x = synth.random_vector(c["A"].shape[0], 77)
        z = host(s.apply(L.MDP_OP_ML, dev(x)))
        zo = c["M"].apply(x)
        scale = np.max(np.abs(zo))
        worst = float(np.max(np.abs(z - zo)) / scale)
        say(f"[fullsize] M_L {prec}: max |dz| / max |z| = {worst:.2e}, global rel {relerr(z, zo):.2e}")
        assert np.all(np.isfinite(z))
        assert worst <= tol
        assert relerr(z, zo) <= tol
    finally:
        s.close()


@pytest.fixture(scope="module")
def cube160(request):
    """The oracle's assembly, hierarchy and FGMRES on one 160^3 system (the
    (K_par, kappa) pair with the fewest iterations).  It runs for a minute or
    more, so its steps are reported past the output capture."""
    capman = request.config.pluginmanager.getplugin("capturemanager")

    def progress(msg):
        with capman.global_and_fixture_disabled():
            say(msg)

    sc = synth.regular_3d(n=160, k_par=1e4, kappa=1e-4, seed=0)
    progress(f"[fullsize] oracle assembly for {sc.name}")
    Ao, bo, po = oa.assemble(sc)
    progress(f"[fullsize] oracle AMG setup (n={Ao.shape[0]})")
    M = osv.setup(Ao, po)
    progress("[fullsize] oracle FGMRES")
    res, _, _ = osv.solve(Ao, bo, po, M=M)
    progress(f"[fullsize] oracle solved in {res.iters} iterations, residual {res.rel_res_true:.2e}")
    A, b, part = tpfa.assemble(sc)
    return {"sc": sc, "Ao": sp.csr_matrix(Ao), "bo": bo, "M": M, "res": res, "A": A, "b": b, "part": part,
            "x": {}}


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec", ["fp64", "mixed"])
def test_cube160_solve_matches_oracle(cube160, prec):
    """160^3 (4.33M unknowns, the launch configuration the benchmark times):
    solution within 1e-6 of the oracle's, iterations within 2, true residual
    of the oracle's matrix at most 1e-8; the error against the oracle is
    reported per precision."""
    c = cube160
    s = Solver(c["A"], c["part"], precision=prec)
    try:
        x, st = s.solve(dev(c["b"]))
        xh = host(x)
        c["x"][prec] = xh
        res = np.linalg.norm(c["bo"] - c["Ao"] @ xh) / np.linalg.norm(c["bo"])
        err = relerr(xh, c["res"].x)
        say(f"[fullsize] 160^3 {prec}: iters {st[0]['iters']} (oracle {c['res'].iters}), residual {res:.2e}, "
            f"error vs oracle {err:.2e}")
        assert st[0]["converged"] == 1
        assert res <= 1e-8
        assert abs(st[0]["iters"] - c["res"].iters) <= 2
        assert err <= 1e-6
    finally:
        s.close()
    if len(c["x"]) == 2:  # mixed against FP64 on the same system
        assert relerr(c["x"]["mixed"], c["x"]["fp64"]) <= 1e-6


@pytest.mark.timeout(900)
@pytest.mark.parametrize("prec,tol", [("fp64", 1e-11), ("mixed", 3e-5)])
def test_cube160_preconditioner_elementwise(cube160, prec, tol):
    """One application of M_L to a seeded vector at 160^3, every one of the
    4.33M outputs against the oracle's."""
    c = cube160
    s = Solver(c["A"], c["part"], precision=prec)
    try:
        x = synth.random_vector(c["A"].shape[0], 78)
        z = host(s.apply(L.MDP_OP_ML, dev(x)))
        zo = c["M"].apply(x)
        worst = float(np.max(np.abs(z - zo)) / np.max(np.abs(zo)))
        say(f"[fullsize] 160^3 M_L {prec}: max |dz| / max |z| = {worst:.2e}, global rel {relerr(z, zo):.2e}")
        assert np.all(np.isfinite(z)) and worst <= tol and relerr(z, zo) <= tol
    finally:
        s.close()
