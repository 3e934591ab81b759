"""Oracle block algebra.  TEST INFRASTRUCTURE ONLY.

* ``split``         the 2x2 host/fracture block structure of eq. (4).
* ``approx_schur``  S~ = A_OO - A_OG diag(A_GG)^{-1} A_GO, eq. (7).
* ``exact_schur_dense``  S = A_OO - A_OG A_GG^{-1} A_GO, eq. (6), dense.

Pins: S~ nonzero pattern equals the unfractured host stencil; with a
diagonal fracture block (no tangential fracture flow) S~ equals the exact S
computed by LAPACK; with no tangential flow S~ equals the closed-form
series-coupled host operator (tests/test_oracle_blocks.py).
"""

from __future__ import annotations

import numpy as np
import scipy.sparse as sp


def split(A, part):
    """Return (omega, gamma, A_OO, A_OG, A_GO, A_GG) with omega/gamma the
    index lists of host (part 0) and fracture (part 1) unknowns in their
    original relative order."""
    part = np.asarray(part)
    omega = np.flatnonzero(part == 0)
    gamma = np.flatnonzero(part == 1)
    A = sp.csr_matrix(A)
    Aoo = A[omega][:, omega].tocsr()
    Aog = A[omega][:, gamma].tocsr()
    Ago = A[gamma][:, omega].tocsr()
    Agg = A[gamma][:, gamma].tocsr()
    return omega, gamma, Aoo, Aog, Ago, Agg


def approx_schur(Aoo, Aog, Ago, Agg):
    """Eq. (7): replace A_GG by its diagonal inside the Schur complement."""
    d = Agg.diagonal()
    S = Aoo - Aog @ sp.diags(1.0 / d) @ Ago
    S = sp.csr_matrix(S)
    S.sum_duplicates()
    S.sort_indices()
    return S


def exact_schur_dense(Aoo, Aog, Ago, Agg):
    """Eq. (6) formed densely (small cases only)."""
    Aoo_d = np.asarray(sp.csr_matrix(Aoo).todense())
    if Agg.shape[0] == 0:
        return Aoo_d
    X = np.linalg.solve(np.asarray(Agg.todense()), np.asarray(Ago.todense()))
    return Aoo_d - np.asarray(Aog.todense()) @ X
