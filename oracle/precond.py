"""Oracle preconditioners.  TEST INFRASTRUCTURE ONLY.

* ``ML``  the inexact block lower-triangular preconditioner M_L of eq. (8),
  applied exactly as Algorithm 1: solve on the host domain with Q_OO
  (V-cycles on S~ of eq. (7)), update the fracture residual with A_GO, solve
  on the fracture block with Q_GG (V-cycles on A_GG), concatenate.
* ``MD`` / ``MU``  the other two block preconditioners that Section 3.2
  derives from the factorisation eq. (5), B_D = D^{-1} and B_U = (U D)^{-1},
  made inexact with the same Q_OO and Q_GG: blocks solved independently, or
  interface first with the domain residual updated by A_OG.
* ``exact_block_lower_dense``  B_L = (D L)^{-1} of Section 3.2 (exact Schur
  complement, exact inverses), and ``approx_block_lower_dense`` B~_L (S~
  with exact inverses), both dense, for the spectral checks of Section 3.2.
* ``block_diag_dense`` / ``block_upper_dense``  B_D = D^{-1} and
  B_U = (U D)^{-1} of Section 3.2, dense.

Pins: M_L, M_D and M_U equal the dense block lower-triangular, diagonal and
upper-triangular solves with the same Q's; with exact blocks (one-level
hierarchies, diagonal fracture block so that S~ = S) M_D and M_U equal the
LAPACK inverses B_D and B_U;
with exact blocks, GMRES converges in at most two iterations because
A B_L = U is unipotent with (U - I)^2 = 0 (Section 3.2 states its
eigenvalues are all one); with a diagonal fracture block the same holds for
B~_L (tests/test_oracle_precond.py).
"""

from __future__ import annotations

from typing import Optional

import numpy as np
import scipy.sparse as sp

from . import amg, blocks


class ML:
    """M_L of eq. (8) with Q_OO, Q_GG = ``cycles`` SA-AMG V-cycles."""

    def __init__(self, A, part, cycles: int = 1, amg_opts: Optional[amg.AMGOptions] = None, labels=None):
        """labels: optional label per unknown of A (the dimension of its
        subdomain) for dimension-aware aggregation on each block's finest level."""
        self.n = A.shape[0]
        (self.omega, self.gamma, self.Aoo, self.Aog,
         self.Ago, self.Agg) = blocks.split(A, part)
        self.S = blocks.approx_schur(self.Aoo, self.Aog, self.Ago, self.Agg)
        self.cycles = cycles
        lo = None if labels is None else np.asarray(labels)[self.omega]
        lg = None if labels is None else np.asarray(labels)[self.gamma]
        self.H_omega = amg.setup(self.S, amg_opts, lo)
        self.H_gamma = amg.setup(self.Agg, amg_opts, lg) if self.gamma.size else None

    def q_omega(self, r):
        return amg.apply_cycles(self.H_omega, r, self.cycles)

    def q_gamma(self, r):
        return amg.apply_cycles(self.H_gamma, r, self.cycles)

    def apply(self, r: np.ndarray) -> np.ndarray:
        """Algorithm 1."""
        r_o = r[self.omega]
        z_o = self.q_omega(r_o)                      # solve in the domain
        z = np.empty_like(r)
        z[self.omega] = z_o
        if self.gamma.size:
            r_g = r[self.gamma] - self.Ago @ z_o     # update the interface residual
            z[self.gamma] = self.q_gamma(r_g)        # solve on the interface
        return z


class MD(ML):
    """Inexact block-diagonal preconditioner: B_D = D^{-1} of Section 3.2
    (D = diag(S, A_GG) from the factorisation eq. (5)) with S^{-1} and
    A_GG^{-1} replaced by the same Q_OO (V-cycles on S~) and Q_GG as M_L.
    The two blocks are solved independently."""

    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.empty_like(r)
        z[self.omega] = self.q_omega(r[self.omega])
        if self.gamma.size:
            z[self.gamma] = self.q_gamma(r[self.gamma])
        return z


class MU(ML):
    """Inexact block upper-triangular preconditioner: B_U = (U D)^{-1} of
    Section 3.2, U D = [[S, A_OG], [0, A_GG]], with the same Q_OO and Q_GG as
    M_L.  Back substitution: solve on the interface, update the domain
    residual with A_OG, solve in the domain."""

    def apply(self, r: np.ndarray) -> np.ndarray:
        z = np.empty_like(r)
        r_o = r[self.omega]
        if self.gamma.size:
            z_g = self.q_gamma(r[self.gamma])        # solve on the interface
            z[self.gamma] = z_g
            r_o = r_o - self.Aog @ z_g               # update the domain residual
        z[self.omega] = self.q_omega(r_o)            # solve in the domain
        return z


FORMS = {"lower": ML, "diag": MD, "upper": MU}


def _dense(M):
    return np.asarray(sp.csr_matrix(M).todense())


def exact_block_lower_dense(A, part):
    """B_L = [[S, 0], [A_GO, A_GG]]^{-1} in the original unknown order."""
    omega, gamma, Aoo, Aog, Ago, Agg = blocks.split(A, part)
    S = blocks.exact_schur_dense(Aoo, Aog, Ago, Agg)
    return _lower_inverse(omega, gamma, S, _dense(Ago), _dense(Agg))


def approx_block_lower_dense(A, part):
    """B~_L = [[S~, 0], [A_GO, A_GG]]^{-1} in the original unknown order."""
    omega, gamma, Aoo, Aog, Ago, Agg = blocks.split(A, part)
    S = _dense(blocks.approx_schur(Aoo, Aog, Ago, Agg))
    return _lower_inverse(omega, gamma, S, _dense(Ago), _dense(Agg))


def _lower_inverse(omega, gamma, S, Ago, Agg):
    n = omega.size + gamma.size
    T = np.zeros((n, n))
    perm = np.concatenate([omega, gamma])
    no = omega.size
    T[:no, :no] = S
    T[no:, :no] = Ago
    T[no:, no:] = Agg
    Tinv = np.linalg.inv(T)
    B = np.zeros((n, n))
    B[np.ix_(perm, perm)] = Tinv
    return B


def block_diag_dense(A, part):
    """B_D = D^{-1} = blockdiag(S, A_GG)^{-1}."""
    omega, gamma, Aoo, Aog, Ago, Agg = blocks.split(A, part)
    S = blocks.exact_schur_dense(Aoo, Aog, Ago, Agg)
    n = omega.size + gamma.size
    B = np.zeros((n, n))
    B[np.ix_(omega, omega)] = np.linalg.inv(S)
    B[np.ix_(gamma, gamma)] = np.linalg.inv(_dense(Agg))
    return B


def block_upper_dense(A, part):
    """B_U = (U D)^{-1} with U D = [[S, A_OG], [0, A_GG]]."""
    omega, gamma, Aoo, Aog, Ago, Agg = blocks.split(A, part)
    S = blocks.exact_schur_dense(Aoo, Aog, Ago, Agg)
    n = omega.size + gamma.size
    no = omega.size
    T = np.zeros((n, n))
    T[:no, :no] = S
    T[:no, no:] = _dense(Aog)
    T[no:, no:] = _dense(Agg)
    perm = np.concatenate([omega, gamma])
    B = np.zeros((n, n))
    B[np.ix_(perm, perm)] = np.linalg.inv(T)
    return B
