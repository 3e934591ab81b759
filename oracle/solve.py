"""Oracle solve phase.  TEST INFRASTRUCTURE ONLY.

``solve`` runs the whole method on an assembled system: split into the
blocks of eq. (4), S~ of eq. (7), SA-AMG setup on S~ and A_GG, and FGMRES
right-preconditioned with M_L (eq. (8), Algorithm 1), zero initial guess.
``solve_dense`` is the LAPACK solution of the same system, the pin for the
whole solve on small cases.

Iteration counts are parity-unpinned against the paper: its Table 1 uses
MPFA on unstructured meshes, Gauss-Seidel smoothing, a 1e-6 tolerance and
benchmark geometries, so its counts are context only.
"""

from __future__ import annotations

import time
from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import amg, fgmres as _fg, precond


@dataclass
class SolveOptions:
    cycles: int = 1
    tol: float = 1e-8
    restart: int = 64
    maxiter: int = 1000
    amg: Optional[amg.AMGOptions] = None
    form: str = "lower"  # block preconditioner: "lower" (M_L), "diag" (M_D) or "upper" (M_U)


def setup(A, part, opts: Optional[SolveOptions] = None, labels=None) -> precond.ML:
    """labels: optional dimension label per unknown (dimension-aware aggregation)."""
    opts = opts or SolveOptions()
    return precond.FORMS[opts.form](sp.csr_matrix(A), part, opts.cycles, opts.amg, labels)


def solve(A, b, part, opts: Optional[SolveOptions] = None, M: Optional[precond.ML] = None,
          x0: Optional[np.ndarray] = None):
    """Return (FGMRESResult, ML, timings dict)."""
    opts = opts or SolveOptions()
    A = sp.csr_matrix(A)
    t0 = time.perf_counter()
    if M is None:
        M = setup(A, part, opts)
    t1 = time.perf_counter()
    res = _fg.fgmres(lambda v: A @ v, b, M.apply, tol=opts.tol, restart=opts.restart,
                     maxiter=opts.maxiter, x0=x0)
    t2 = time.perf_counter()
    return res, M, {"setup_s": t1 - t0, "solve_s": t2 - t1}


def solve_dense(A, b) -> np.ndarray:
    return np.linalg.solve(np.asarray(sp.csr_matrix(A).todense()), np.asarray(b, dtype=np.float64))
