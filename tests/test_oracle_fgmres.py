"""Pins of the oracle flexible GMRES (right preconditioning, Section 3.2;
zero initial guess and relative-residual stop, Section 4)."""

import numpy as np
import pytest

from oracle.fgmres import fgmres


def _matrix(n, seed, sym=False):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((n, n)) / np.sqrt(n) + 2.0 * np.eye(n)
    if sym:
        A = A @ A.T + np.eye(n)
    return A


def _krylov_min_residual(A, b, k):
    """Brute force: min_y ||b - A K_k y|| over K_k = span{b, Ab, ...}."""
    K = [b / np.linalg.norm(b)]
    for _ in range(k - 1):
        v = A @ K[-1]
        for u in K:  # two passes keep the basis orthonormal enough
            v = v - (u @ v) * u
        for u in K:
            v = v - (u @ v) * u
        K.append(v / np.linalg.norm(v))
    Kk = np.column_stack(K)
    y, *_ = np.linalg.lstsq(A @ Kk, b, rcond=None)
    return np.linalg.norm(b - A @ Kk @ y)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_identity_preconditioner_minimises_residual(seed):
    n = 40
    A = _matrix(n, seed)
    b = np.random.default_rng(seed + 10).standard_normal(n)
    res = fgmres(lambda v: A @ v, b, None, tol=1e-13, restart=64)
    for k in range(1, 9):
        expect = _krylov_min_residual(A, b, k) / np.linalg.norm(b)
        assert abs(res.history[k - 1] - expect) <= 1e-9 * max(expect, 1e-3)


def test_exact_inverse_preconditioner_one_step():
    A = _matrix(30, 3)
    Ainv = np.linalg.inv(A)
    b = np.random.default_rng(4).standard_normal(30)
    res = fgmres(lambda v: A @ v, b, lambda v: Ainv @ v, tol=1e-10)
    assert res.converged and res.iters == 1


def test_dense_converges_within_n_steps():
    n = 14
    A = _matrix(n, 5)
    b = np.random.default_rng(6).standard_normal(n)
    res = fgmres(lambda v: A @ v, b, None, tol=1e-10, restart=64)
    assert res.converged and res.iters <= n
    assert np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)


def test_lucky_breakdown():
    """b lies in a 2-dimensional invariant subspace: the Krylov space stops
    growing at step 2 and the solution is exact there."""
    A = np.diag([1.0, 3.0, 5.0, 7.0])
    b = np.array([1.0, 1.0, 0.0, 0.0])
    res = fgmres(lambda v: A @ v, b, None, tol=1e-14)
    assert res.converged and res.iters == 2
    assert np.allclose(res.x, [1.0, 1.0 / 3.0, 0.0, 0.0], atol=1e-14)


def test_restarted_run_reaches_tolerance():
    n = 60
    A = _matrix(n, 7, sym=True)
    b = np.random.default_rng(8).standard_normal(n)
    res = fgmres(lambda v: A @ v, b, None, tol=1e-10, restart=5, maxiter=500)
    assert res.converged and res.restarts >= 1
    assert np.linalg.norm(b - A @ res.x) <= 1e-10 * np.linalg.norm(b)


def test_zero_rhs_and_iteration_budget():
    A = _matrix(10, 9)
    res = fgmres(lambda v: A @ v, np.zeros(10), None)
    assert res.converged and res.iters == 0 and not res.x.any()
    b = np.random.default_rng(1).standard_normal(10)
    res = fgmres(lambda v: A @ v, b, None, tol=1e-14, maxiter=3)
    assert not res.converged and res.iters == 3


def test_flexible_variable_preconditioner():
    """A preconditioner that changes every step (flexible GMRES keeps Z):
    the returned x still has the residual the method reports."""
    A = _matrix(25, 11, sym=True)
    b = np.random.default_rng(12).standard_normal(25)
    state = {"k": 0}

    def M(v):
        state["k"] += 1
        return v / (1.0 + 0.3 * np.sin(state["k"]))

    res = fgmres(lambda v: A @ v, b, M, tol=1e-10)
    assert res.converged
    assert np.linalg.norm(b - A @ res.x) / np.linalg.norm(b) == pytest.approx(res.rel_res_true)
