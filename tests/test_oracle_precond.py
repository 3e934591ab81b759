"""Pins of the oracle preconditioners: M_L (eq. (8)) applied by Algorithm 1,
and the exact block preconditioners of Section 3.2."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import Fracture, Scenario
from oracle import amg, precond, solve as osv
from oracle import assembly as oa
from oracle.fgmres import fgmres


def _op(f, n):
    return np.column_stack([f(e) for e in np.eye(n)])


@pytest.mark.parametrize("make", [lambda: synth.tiny_2d(8, seed=1), lambda: synth.tiny_3d(5, seed=2)])
@pytest.mark.parametrize("cycles", [1, 2])
def test_algorithm1_equals_eq8(make, cycles):
    """Algorithm 1 computes z = M_L r with M_L^{-1} = [[Q_OO^{-1}, 0],
    [A_GO, Q_GG^{-1}]] (eq. (8)); checked densely with the Q's extracted as
    operators."""
    A, b, part = oa.assemble(make())
    M = precond.ML(A, part, cycles=cycles, amg_opts=amg.AMGOptions(max_coarse=8))
    n = A.shape[0]
    no, ng = M.omega.size, M.gamma.size
    Qo = _op(M.q_omega, no)
    Qg = _op(M.q_gamma, ng)
    Minv = np.zeros((n, n))
    Minv[:no, :no] = np.linalg.inv(Qo)
    Minv[no:, :no] = M.Ago.toarray()
    Minv[no:, no:] = np.linalg.inv(Qg)
    ML = _op(M.apply, n)
    assert np.allclose(ML, np.linalg.inv(Minv), atol=1e-10 * np.abs(ML).max())


def test_multiple_cycles_are_stationary_iteration():
    A, b, part = oa.assemble(synth.tiny_2d(12, seed=5))
    M1 = precond.ML(A, part, cycles=1, amg_opts=amg.AMGOptions(max_coarse=8))
    M3 = precond.ML(A, part, cycles=3, amg_opts=amg.AMGOptions(max_coarse=8))
    r = synth.random_vector(M1.S.shape[0], 3)
    V = lambda v: M1.q_omega(v)
    z = V(r)
    z = z + V(r - M1.S @ z)
    z = z + V(r - M1.S @ z)
    assert np.allclose(M3.q_omega(r), z, rtol=1e-13, atol=1e-15)


@pytest.mark.parametrize("make", [lambda: synth.tiny_2d(8), lambda: synth.tiny_3d(4, seed=3),
                                  lambda: synth.grid_2d_four_lines(12, 1e4, 1e-4)])
def test_exact_block_lower_two_iterations(make):
    """A B_L = U (Section 3.2): unipotent, (U - I)^2 = 0, so GMRES needs at
    most two steps."""
    A, b, part = oa.assemble(make())
    B = precond.exact_block_lower_dense(A, part)
    Ad = A.toarray()
    N = Ad @ B - np.eye(A.shape[0])
    assert np.abs(N @ N).max() <= 1e-8 * max(1.0, np.abs(N).max() ** 2)
    res = fgmres(lambda v: A @ v, b, lambda v: B @ v, tol=1e-10)
    assert res.converged and res.iters <= 2


def test_block_factorisation_and_upper_variant():
    """Eq. (5): A = U D L with U = [[I, A_OG A_GG^-1], [0, I]], D = diag(S, A_GG),
    L = [[I, 0], [A_GG^-1 A_GO, I]].  B_D = D^{-1} inverts D exactly, and
    A B_U = (U D) L (U D)^{-1} is similar to the unipotent L, so GMRES with
    B_U needs at most two steps."""
    A, b, part = oa.assemble(synth.tiny_2d(8, seed=4))
    from oracle import blocks as ob
    omega, gamma, Aoo, Aog, Ago, Agg = ob.split(A, part)
    no, ng = omega.size, gamma.size
    Gi = np.linalg.inv(Agg.toarray())
    S = ob.exact_schur_dense(Aoo, Aog, Ago, Agg)
    U = np.eye(no + ng); U[:no, no:] = Aog.toarray() @ Gi
    L = np.eye(no + ng); L[no:, :no] = Gi @ Ago.toarray()
    D = np.zeros((no + ng, no + ng)); D[:no, :no] = S; D[no:, no:] = Agg.toarray()
    assert np.allclose(U @ D @ L, A.toarray(), atol=1e-12 * np.abs(A).max())
    Bd = precond.block_diag_dense(A, part)
    assert np.allclose(Bd @ D, np.eye(no + ng), atol=1e-10)
    Bu = precond.block_upper_dense(A, part)
    res = fgmres(lambda v: A @ v, b, lambda v: Bu @ v, tol=1e-10)
    assert res.converged and res.iters <= 2


def test_approx_block_lower_exact_when_fracture_block_diagonal():
    n = 8
    fr = [Fracture(0, 2, (1,), (2,), 3.0, 0.5, 1e-2), Fracture(1, 5, (4,), (5,), 1.0, 4.0, 1e-3)]
    sc = Scenario(2, n, np.ones(n * n), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = oa.assemble(sc)
    B = precond.approx_block_lower_dense(A, part)
    res = fgmres(lambda v: A @ v, b, lambda v: B @ v, tol=1e-10)
    assert res.converged and res.iters <= 2


@pytest.mark.parametrize("make", [lambda: synth.grid_2d_four_lines(32),
                                  lambda: synth.regular_3d(n=8, seed=1),
                                  lambda: synth.regular_3d(n=8, k_par=1e-4, kappa=1e4, seed=2)])
def test_whole_solve_matches_lapack(make):
    A, b, part = oa.assemble(make())
    res, M, _ = osv.solve(A, b, part)
    x = osv.solve_dense(A, b)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) <= 1e-8 * np.linalg.norm(b)
    cond = np.linalg.cond(A.toarray())
    err = np.linalg.norm(res.x - x) / np.linalg.norm(x)
    assert err <= cond * 1e-8


@pytest.mark.parametrize("make", [lambda: synth.tiny_2d(8, seed=1), lambda: synth.tiny_3d(5, seed=2)])
def test_diag_and_upper_forms_equal_their_block_solves(make):
    """M_D^{-1} = blockdiag(Q_OO^{-1}, Q_GG^{-1}) and
    M_U^{-1} = [[Q_OO^{-1}, A_OG], [0, Q_GG^{-1}]] (Section 3.2 with the
    inexact blocks of eq. (8)); checked densely with the Q's as operators."""
    A, b, part = oa.assemble(make())
    opts = amg.AMGOptions(max_coarse=8)
    MD = precond.MD(A, part, amg_opts=opts)
    MU = precond.MU(A, part, amg_opts=opts)
    n = A.shape[0]
    no = MD.omega.size
    Qo, Qg = _op(MD.q_omega, no), _op(MD.q_gamma, n - no)
    perm = np.concatenate([MD.omega, MD.gamma])
    Dinv = np.zeros((n, n))
    Dinv[:no, :no] = np.linalg.inv(Qo)
    Dinv[no:, no:] = np.linalg.inv(Qg)
    Uinv = Dinv.copy()
    Uinv[:no, no:] = MU.Aog.toarray()
    for M, Minv in ((MD, Dinv), (MU, Uinv)):
        Z = _op(M.apply, n)[np.ix_(perm, perm)]
        assert np.allclose(Z, np.linalg.inv(Minv), atol=1e-10 * np.abs(Z).max())


def test_diag_and_upper_forms_exact_blocks():
    """With one-level hierarchies (Q = exact inverses) and no tangential
    fracture flow (A_GG diagonal, so S~ = S), M_D and M_U are exactly the
    B_D = D^{-1} and B_U = (U D)^{-1} of Section 3.2, computed by LAPACK;
    B_U then needs at most two GMRES steps."""
    n = 8
    fr = [Fracture(0, 2, (1,), (2,), 3.0, 0.5, 1e-2), Fracture(1, 5, (4,), (5,), 1.0, 4.0, 1e-3)]
    sc = Scenario(2, n, np.ones(n * n), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = oa.assemble(sc)
    exact = amg.AMGOptions(max_coarse=10 ** 6)
    N = A.shape[0]
    for cls, dense in ((precond.MD, precond.block_diag_dense), (precond.MU, precond.block_upper_dense)):
        M = cls(A, part, amg_opts=exact)
        assert len(M.H_omega.levels) == 1
        B = dense(A, part)
        assert np.allclose(_op(M.apply, N), B, atol=1e-10 * np.abs(B).max())
    res = fgmres(lambda v: A @ v, b, precond.MU(A, part, amg_opts=exact).apply, tol=1e-10)
    assert res.converged and res.iters <= 2


@pytest.mark.parametrize("form", ["diag", "upper"])
def test_diag_and_upper_solves_match_lapack(form):
    A, b, part = oa.assemble(synth.regular_3d(n=8, seed=1))
    res, _, _ = osv.solve(A, b, part, osv.SolveOptions(form=form))
    x = osv.solve_dense(A, b)
    assert res.converged and res.rel_res_true <= 1e-8
    assert np.linalg.norm(res.x - x) <= 1e-6 * np.linalg.norm(x)
