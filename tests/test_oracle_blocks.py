"""Pins of the oracle block algebra: eq. (4) split, eq. (6) exact Schur
complement and eq. (7) approximate Schur complement."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import Fracture, Scenario
from oracle import assembly as oa
from oracle import blocks as ob


def _host_stencil_pattern(n, dim):
    """Pattern of the unfractured host 5/7-point stencil."""
    N = n ** dim
    rows, cols = list(range(N)), list(range(N))
    for c in range(N):
        coords = [(c // n ** a) % n for a in range(dim)]
        for a in range(dim):
            for s in (-1, 1):
                q = coords[a] + s
                if 0 <= q < n:
                    rows.append(c)
                    cols.append(c + s * n ** a)
    return sp.csr_matrix((np.ones(len(rows)), (rows, cols)), shape=(N, N))


@pytest.mark.parametrize("make", [
    lambda: synth.grid_2d_four_lines(32),
    lambda: synth.tiny_2d(12, seed=1),
    lambda: synth.regular_3d(n=8, seed=2),
    lambda: synth.tiny_3d(7, seed=5),
])
def test_approx_schur_pattern_is_host_stencil(make):
    """Eliminating each fracture cell through its diagonal reconnects the two
    host cells of its face, so S~ has exactly the unfractured host pattern."""
    sc = make()
    A, b, part = oa.assemble(sc)
    _, _, Aoo, Aog, Ago, Agg = ob.split(A, part)
    S = ob.approx_schur(Aoo, Aog, Ago, Agg)
    P = _host_stencil_pattern(sc.n, sc.dim)
    assert S.nnz == P.nnz
    assert ((S != 0).astype(int) != (P != 0).astype(int)).nnz == 0


def _isolated_cells(dim, n=8):
    """Single-cell fractures far apart: no two fracture cells share a
    facet, so A_GG is diagonal."""
    if dim == 2:
        fr = [Fracture(0, 2, (1,), (2,), 3.0, 0.5, 1e-2),
              Fracture(1, 5, (4,), (5,), 1.0, 4.0, 1e-3),
              Fracture(0, 6, (6,), (7,), 10.0, 1e-2, 1e-2)]
    else:
        fr = [Fracture(0, 2, (1, 1), (2, 2), 3.0, 0.5, 1e-2),
              Fracture(1, 5, (4, 5), (5, 6), 1.0, 4.0, 1e-3),
              Fracture(2, 4, (6, 2), (7, 3), 10.0, 1e-2, 1e-2)]
    k = np.exp(np.random.default_rng(dim).standard_normal(n ** dim))
    return Scenario(dim, n, k, fr, {(0, 0): 1.0, (0, 1): 0.0})


@pytest.mark.parametrize("dim", [2, 3])
def test_approx_schur_equals_exact_when_fracture_block_diagonal(dim):
    A, b, part = oa.assemble(_isolated_cells(dim))
    _, _, Aoo, Aog, Ago, Agg = ob.split(A, part)
    assert sp.triu(Agg, 1).nnz == 0  # precondition: A_GG diagonal
    S_t = ob.approx_schur(Aoo, Aog, Ago, Agg).toarray()
    S = ob.exact_schur_dense(Aoo, Aog, Ago, Agg)  # LAPACK solve
    assert np.allclose(S_t, S, rtol=1e-14, atol=1e-14 * np.abs(S).max())


def test_approx_schur_series_closed_form():
    """No tangential fracture flow (isolated cells): the S~ coupling across a
    fractured face is the series combination of the host half cells and the
    normal resistance of eq. (2): -1/(1/t_L + 1/t_R + a/(kappa A))."""
    sc = _isolated_cells(2)
    n, h = sc.n, 1.0 / sc.n
    A, b, part = oa.assemble(sc)
    _, _, Aoo, Aog, Ago, Agg = ob.split(A, part)
    S = ob.approx_schur(Aoo, Aog, Ago, Agg).toarray()
    t = 2.0 * sc.k_host * h / h
    for fr in sc.fractures:
        j = fr.lo[0]
        if fr.axis == 0:
            L, R = (fr.index - 1) + n * j, fr.index + n * j
        else:
            L, R = j + n * (fr.index - 1), j + n * fr.index
        expect = -1.0 / (1.0 / t[L] + 1.0 / t[R] + fr.aperture / (fr.kappa * h))
        assert abs(S[L, R] - expect) < 1e-14 * abs(expect)
        assert S[L, R] == S[R, L]


def test_split_preserves_order_and_roundtrip():
    sc = synth.tiny_2d(8)
    A, b, part = oa.assemble(sc)
    # scramble the unknown order, then split: blocks must be those of the
    # unscrambled system
    perm = np.random.default_rng(0).permutation(A.shape[0])
    Ap = A[perm][:, perm]
    omega, gamma, Aoo, Aog, Ago, Agg = ob.split(Ap, part[perm])
    _, _, Aoo0, Aog0, Ago0, Agg0 = ob.split(A, part)
    inv_o = perm[omega]
    assert np.all(np.diff(omega) > 0)
    assert (Aoo != A[inv_o][:, inv_o]).nnz == 0
    # with the natural ordering the blocks are contiguous
    assert Aoo0.shape[0] == sc.n_host
