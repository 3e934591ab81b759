"""Oracle flexible GMRES.  TEST INFRASTRUCTURE ONLY.

Right-preconditioned GMRES is what Section 3.2 analyses (A B_L), and the
experiments of Section 4 start from a zero initial guess and stop on the
relative residual.  Because the preconditioner (AMG V-cycles) is applied
as a procedure, the flexible variant (Saad 1993, SIAM J. Sci. Comput.
14(2)) is used: the preconditioned directions z_j are kept and the update is
x = x0 + Z y.  Arnoldi uses modified Gram-Schmidt, the least-squares problem
is reduced with Givens rotations, and a cycle ends when the estimated
residual |g_{j+1}| drops to tol * ||b||, on a lucky breakdown, or after
``restart`` steps.  After each cycle the true residual b - A x is formed;
the solve ends when it meets tol * ||b|| (or the iteration budget is spent),
otherwise a new cycle starts from x.  The iteration count is the number of
preconditioner applications.

Pins: with the identity preconditioner the residual after k steps equals
the brute-force least-squares minimum over the Krylov space; with the exact
inverse as preconditioner one step suffices; a dense n x n system converges
in at most n steps; a lucky breakdown returns a converged result
(tests/test_oracle_fgmres.py).
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Callable, List, Optional

import numpy as np


@dataclass
class FGMRESResult:
    x: np.ndarray
    iters: int
    restarts: int
    converged: bool
    rel_res_true: float
    rel_res_est: float
    history: List[float] = field(default_factory=list)  # estimated rel. residual per step


def fgmres(matvec: Callable, b: np.ndarray, precond: Optional[Callable] = None,
           tol: float = 1e-8, restart: int = 64, maxiter: int = 1000,
           x0: Optional[np.ndarray] = None) -> FGMRESResult:
    b = np.asarray(b, dtype=np.float64)
    n = b.shape[0]
    M = precond if precond is not None else (lambda v: v.copy())
    bnorm = float(np.linalg.norm(b))
    x = np.zeros(n) if x0 is None else np.array(x0, dtype=np.float64)
    if bnorm == 0.0:
        return FGMRESResult(np.zeros(n), 0, 0, True, 0.0, 0.0, [])
    iters = 0
    cycles = 0
    history: List[float] = []
    est = np.inf
    while True:
        r = b - matvec(x)
        beta = float(np.linalg.norm(r))
        true_rel = beta / bnorm
        if true_rel <= tol or iters >= maxiter:
            return FGMRESResult(x, iters, max(cycles - 1, 0), true_rel <= tol, true_rel,
                                est if np.isfinite(est) else true_rel, history)
        m = restart
        V = np.zeros((m + 1, n))
        Z = np.zeros((m, n))
        H = np.zeros((m + 1, m))
        cs = np.zeros(m)
        sn = np.zeros(m)
        g = np.zeros(m + 1)
        g[0] = beta
        V[0] = r / beta
        k = 0
        for j in range(m):
            Z[j] = M(V[j])
            iters += 1
            w = matvec(Z[j])
            for i in range(j + 1):           # modified Gram-Schmidt
                H[i, j] = float(V[i] @ w)
                w = w - H[i, j] * V[i]
            wnorm = float(np.linalg.norm(w))
            H[j + 1, j] = wnorm
            for i in range(j):               # previous rotations
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = float(np.hypot(H[j, j], H[j + 1, j]))
            breakdown = H[j + 1, j] == 0.0
            cs[j] = H[j, j] / den
            sn[j] = H[j + 1, j] / den
            H[j, j] = den
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            H[j + 1, j] = 0.0
            est = abs(g[j + 1]) / bnorm
            history.append(est)
            k = j + 1
            if breakdown or est <= tol or iters >= maxiter:
                break
            V[j + 1] = w / wnorm
        y = np.zeros(k)
        for i in range(k - 1, -1, -1):       # back substitution
            y[i] = (g[i] - H[i, i + 1:k] @ y[i + 1:k]) / H[i, i]
        x = x + Z[:k].T @ y
        cycles += 1
