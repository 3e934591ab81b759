"""Oracle smoothed-aggregation AMG.  TEST INFRASTRUCTURE ONLY.

Section 3.3 defines Q_OmegaOmega and Q_GammaGamma as V-cycles of
smoothed-aggregation AMG (Vanek, Mandel, Brezina 1996) on S~ and A_GG, one
cycle by default with the cycle count adjustable.  The paper does not fix
the SA parameters or the smoother for this library's setting, so the
following reading is used (every rule below is deterministic):

* strength: j != i is a strong neighbour of i iff
  |a_ij| >= theta * sqrt(|a_ii a_jj|), theta = 0.02 on every level (with
  0.08 the iteration counts grew with the grid, 82 at 100^3 and 156 at
  160^3 on the hardest regular systems; 0.02 keeps most couplings of the
  log-normal host strong, and 20-60 iterations from 50^3 to 160^3);
* dimension-aware aggregation (Section 3.3, last paragraph: aggregates
  built inside subdomains of one dimension first, crossing dimensions only
  later): when the finest level's unknowns carry labels (the dimension of
  their subdomain), a strong neighbour must also carry the same label there;
  coarser levels are not restricted;
* aggregation in natural order.  Pass 1: a node with at least one strong
  neighbour that is itself unaggregated and whose strong neighbours are all
  unaggregated starts a new aggregate {i} + N_i.  Pass 2: every remaining
  node with strong neighbours joins the pass-1 aggregate of its lowest-index
  strong neighbour that pass 1 aggregated (labels as left by pass 1).
  Pass 3: every still-unaggregated node with strong neighbours starts a new
  aggregate with its still-unaggregated strong neighbours.  Nodes without
  strong neighbours stay unaggregated (zero tentative row);
* tentative prolongator: aggregate indicator columns scaled to unit 2-norm;
* smoothed prolongator P = (I - omega D^{-1} A) P_tent with D = diag(A),
  omega = (4/3) / rho, rho = max_i sum_j |a_ij| / |a_ii| (Gershgorin);
* R = P^T, A_c = R A P;
* coarsening stops when n <= max_coarse (400), no aggregate forms, the
  coarse size exceeds 0.9 n, or the hierarchy reaches max_levels (10);
* the coarsest level is solved exactly (dense LAPACK) when n <= max_dense
  (2000), else by four l1-Jacobi sweeps from zero;
* smoother: l1-Jacobi (Baker, Falgout, Kolev, Yang 2011) with one-row
  blocks, d_i = sum_j |a_ij|, undamped; one sweep before (from a zero
  guess, so x = b / d) and one after the coarse correction.  Section 4 uses
  one smoothing step on each side; the counts are options (pre_sweeps,
  post_sweeps), each further sweep being x <- x + (b - A x) / d;
* smoother option "gs": the Gauss-Seidel smoothing of Section 4 in
  multicolour form.  Each level is coloured greedily in natural order (node
  i takes the smallest colour not taken by an already coloured neighbour in
  the symmetrised pattern); a forward sweep updates the colours in
  increasing order, x_i = (b_i - sum_{j != i} a_ij x_j) / a_ii for every
  node of the colour at once (nodes of one colour are not coupled), which
  is Gauss-Seidel in the order (colour, index); pre-smoothing is forward
  sweeps from zero, post-smoothing backward sweeps (colours in decreasing
  order), so the cycle stays symmetric for a symmetric matrix.  The
  swept coarsest level keeps its l1-Jacobi sweeps.

Pins: tentative columns orthonormal; coarse operators symmetric; constant
vector preserved on a pure-Neumann graph; one-level hierarchy is an exact
solve; a two-level cycle equals the textbook two-grid error propagator; a
V-cycle of any depth, with any sweep counts and a dense or swept coarsest
level, equals the operator of the textbook multigrid recursion
B_l = (I - E_l) A_l^-1, E_l = S_l^post (I - P B_{l+1} R A_l) S_l^pre with
S_l = I - D_l^-1 A_l; k l1-Jacobi sweeps from zero equal
(I - S^k) A^-1 b; nu cycles as a stationary iteration equal
(I - E_0^nu) A^-1 b; the V-cycle operator is symmetric positive definite; hand-computed aggregates
on small graphs (tests/test_oracle_amg.py, tests/golden/).  Multicolour
Gauss-Seidel: colourings valid and equal to hand-computed ones on a chain
and a grid (red-black); one forward (backward) sweep equals the dense
triangular solve (D + L)^-1 (b - U x) ((D + U)^-1 (b - L x)) in the
(colour, index) order; the cycle equals the multigrid recursion with those
smoothing matrices and is symmetric.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class AMGOptions:
    theta: float = 0.02
    max_coarse: int = 400
    max_dense: int = 2000
    max_levels: int = 10
    coarse_sweeps: int = 4
    pre_sweeps: int = 1
    post_sweeps: int = 1
    smoother: str = "l1jacobi"  # or "gs": multicolour Gauss-Seidel


@dataclass
class Level:
    A: sp.csr_matrix
    d_l1: np.ndarray
    P: Optional[sp.csr_matrix] = None
    R: Optional[sp.csr_matrix] = None
    agg: Optional[np.ndarray] = None
    colour: Optional[np.ndarray] = None  # multicolour Gauss-Seidel


def greedy_colours(A) -> np.ndarray:
    """Colour per node: in natural order, the smallest colour not used by an
    already coloured neighbour (pattern of A + A^T, diagonal excluded)."""
    A = sp.csr_matrix(A)
    G = sp.csr_matrix(abs(A) + abs(A.T))
    n = A.shape[0]
    col = np.full(n, -1, dtype=np.int64)
    for i in range(n):
        used = set()
        for p in range(G.indptr[i], G.indptr[i + 1]):
            j = int(G.indices[p])
            if j != i and col[j] >= 0:
                used.add(int(col[j]))
        c = 0
        while c in used:
            c += 1
        col[i] = c
    return col


def gs_sweep(A, b: np.ndarray, x: np.ndarray, colour: np.ndarray, forward: bool) -> np.ndarray:
    """One multicolour Gauss-Seidel sweep (colours ascending if forward)."""
    A = sp.csr_matrix(A)
    d = A.diagonal()
    x = x.copy()
    order = range(int(colour.max()) + 1) if forward else range(int(colour.max()), -1, -1)
    for c in order:
        idx = np.flatnonzero(colour == c)
        off = A[idx] @ x - d[idx] * x[idx]
        x[idx] = (b[idx] - off) / d[idx]
    return x


@dataclass
class Hierarchy:
    levels: List[Level] = field(default_factory=list)
    coarse_dense: Optional[np.ndarray] = None  # coarsest matrix when solved exactly
    opts: AMGOptions = field(default_factory=AMGOptions)

    def sizes(self):
        return [lv.A.shape[0] for lv in self.levels]


def l1_diagonal(A) -> np.ndarray:
    """d_i = sum_j |a_ij|."""
    return np.asarray(abs(sp.csr_matrix(A)).sum(axis=1)).ravel()


def strong_neighbours(A, theta: float, labels=None):
    """Per row, the ascending list of strong neighbours (see module header);
    with labels, only neighbours of the same label."""
    A = sp.csr_matrix(A)
    diag = A.diagonal()
    out = []
    for i in range(A.shape[0]):
        lo, hi = A.indptr[i], A.indptr[i + 1]
        row = []
        for p in range(lo, hi):
            j = int(A.indices[p])
            if j == i or (labels is not None and labels[j] != labels[i]):
                continue
            if abs(A.data[p]) >= theta * np.sqrt(abs(diag[i] * diag[j])):
                row.append(j)
        row.sort()
        out.append(row)
    return out


def aggregate(strong):
    """Three-pass greedy aggregation in natural order.  Returns (agg, n_agg)
    with agg[i] = -1 for nodes left out."""
    n = len(strong)
    agg = [-1] * n
    n_agg = 0
    for i in range(n):  # pass 1
        nb = strong[i]
        if not nb or agg[i] != -1:
            continue
        if any(agg[j] != -1 for j in nb):
            continue
        agg[i] = n_agg
        for j in nb:
            agg[j] = n_agg
        n_agg += 1
    after_pass1 = list(agg)
    for i in range(n):  # pass 2
        if agg[i] != -1 or not strong[i]:
            continue
        for j in strong[i]:
            if after_pass1[j] != -1:
                agg[i] = after_pass1[j]
                break
    for i in range(n):  # pass 3
        if agg[i] != -1 or not strong[i]:
            continue
        agg[i] = n_agg
        for j in strong[i]:
            if agg[j] == -1:
                agg[j] = n_agg
        n_agg += 1
    return np.array(agg, dtype=np.int64), n_agg


def tentative(agg: np.ndarray, n_agg: int) -> sp.csr_matrix:
    n = agg.shape[0]
    sizes = np.bincount(agg[agg >= 0], minlength=n_agg).astype(np.float64)
    rows = np.flatnonzero(agg >= 0)
    cols = agg[rows]
    vals = 1.0 / np.sqrt(sizes[cols])
    return sp.csr_matrix((vals, (rows, cols)), shape=(n, n_agg))


def smoothed_prolongator(A, P_tent):
    A = sp.csr_matrix(A)
    diag = A.diagonal()
    rho = float(np.max(l1_diagonal(A) / np.abs(diag)))
    omega = (4.0 / 3.0) / rho
    P = P_tent - omega * (sp.diags(1.0 / diag) @ (A @ P_tent))
    P = sp.csr_matrix(P)
    P.sum_duplicates()
    P.sort_indices()
    return P


def setup(A, opts: Optional[AMGOptions] = None, labels=None) -> Hierarchy:
    """labels: optional label per unknown of A (dimension-aware aggregation
    on the finest level)."""
    opts = opts or AMGOptions()
    H = Hierarchy(opts=opts)
    Acur = sp.csr_matrix(A)
    while True:
        n = Acur.shape[0]
        lv = Level(A=Acur, d_l1=l1_diagonal(Acur))
        if opts.smoother == "gs":
            lv.colour = greedy_colours(Acur)
        H.levels.append(lv)
        if n <= opts.max_coarse or len(H.levels) >= opts.max_levels:
            break
        agg, n_agg = aggregate(strong_neighbours(Acur, opts.theta, labels if len(H.levels) == 1 else None))
        if n_agg == 0 or n_agg > 0.9 * n:
            break
        P = smoothed_prolongator(Acur, tentative(agg, n_agg))
        R = sp.csr_matrix(P.T)
        Ac = sp.csr_matrix(R @ Acur @ P)
        Ac.sum_duplicates()
        Ac.sort_indices()
        lv.P, lv.R, lv.agg = P, R, agg
        Acur = Ac
    last = H.levels[-1]
    if last.A.shape[0] <= opts.max_dense:
        H.coarse_dense = np.asarray(last.A.todense())
    return H


def _coarse_solve(H: Hierarchy, b: np.ndarray) -> np.ndarray:
    last = H.levels[-1]
    if H.coarse_dense is not None:
        if b.shape[0] == 0:
            return b.copy()
        return np.linalg.solve(H.coarse_dense, b)
    x = b / last.d_l1
    for _ in range(H.opts.coarse_sweeps - 1):
        x = x + (b - last.A @ x) / last.d_l1
    return x


def vcycle(H: Hierarchy, b: np.ndarray, lvl: int = 0) -> np.ndarray:
    """One V-cycle from a zero initial guess."""
    if lvl == len(H.levels) - 1:
        return _coarse_solve(H, b)
    lv = H.levels[lvl]
    gs = H.opts.smoother == "gs"
    if gs:                               # pre-smoothing: forward sweeps from zero
        x = np.zeros_like(b)
        for _ in range(H.opts.pre_sweeps):
            x = gs_sweep(lv.A, b, x, lv.colour, True)
    else:
        x = b / lv.d_l1                  # pre-smoothing from zero
        for _ in range(H.opts.pre_sweeps - 1):
            x = x + (b - lv.A @ x) / lv.d_l1
    r = b - lv.A @ x
    xc = vcycle(H, lv.R @ r, lvl + 1)   # coarse-grid correction
    x = x + lv.P @ xc
    for _ in range(H.opts.post_sweeps):  # post-smoothing
        x = gs_sweep(lv.A, b, x, lv.colour, False) if gs else x + (b - lv.A @ x) / lv.d_l1
    return x


def apply_cycles(H: Hierarchy, b: np.ndarray, cycles: int = 1) -> np.ndarray:
    """``cycles`` V-cycles as a stationary iteration from zero."""
    x = vcycle(H, b)
    A = H.levels[0].A
    for _ in range(cycles - 1):
        x = x + vcycle(H, b - A @ x)
    return x
