"""Pins of the oracle smoothed-aggregation AMG (Section 3.3 reading)."""

import os

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from oracle import amg
from oracle import assembly as oa
from oracle import blocks as ob

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _golden(name):
    data = np.loadtxt(os.path.join(GOLDEN, name), comments="#", dtype=np.int64)
    return data[:, 1]


def _chain(n):
    A = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1]).tolil()
    A[0, 0] = A[n - 1, n - 1] = 1.0
    return A.tocsr()


def _grid(m):
    T = sp.diags([-np.ones(m - 1), 2 * np.ones(m), -np.ones(m - 1)], [-1, 0, 1])
    I = sp.identity(m)
    return sp.csr_matrix(sp.kron(I, T) + sp.kron(T, I))


def _weak_star():
    A = 10.0 * np.eye(5)
    for i, j, v in [(0, 1, -5.0), (1, 2, -0.5), (2, 3, -5.0), (3, 4, -5.0)]:
        A[i, j] = A[j, i] = v
    return sp.csr_matrix(A)


def _pass2_graph():
    edges = [(0, 1), (1, 2), (2, 5), (3, 4), (4, 5)]
    A = np.zeros((6, 6))
    for i, j in edges:
        A[i, j] = A[j, i] = -1.0
    A[np.diag_indices(6)] = -A.sum(axis=1) + 1.0
    return sp.csr_matrix(A)


@pytest.mark.parametrize("name,make", [
    ("aggregation_pass2_snapshot.txt", _pass2_graph),
    ("aggregation_chain7.txt", lambda: _chain(7)),
    ("aggregation_grid4x4.txt", lambda: _grid(4)),
    ("aggregation_weak_star.txt", _weak_star),
])
def test_aggregates_match_hand_computation(name, make):
    agg, n_agg = amg.aggregate(amg.strong_neighbours(make(), 0.08))
    assert np.array_equal(agg, _golden(name))
    assert n_agg == int(_golden(name).max()) + 1


def test_node_without_strong_neighbours_stays_out():
    A = np.array([[10.0, -0.1, 0.0], [-0.1, 2.0, -1.0], [0.0, -1.0, 2.0]])
    agg, n_agg = amg.aggregate(amg.strong_neighbours(sp.csr_matrix(A), 0.08))
    assert agg[0] == -1 and agg[1] == agg[2] == 0 and n_agg == 1


def _system_blocks(sc):
    A, b, part = oa.assemble(sc)
    _, _, Aoo, Aog, Ago, Agg = ob.split(A, part)
    return ob.approx_schur(Aoo, Aog, Ago, Agg), Agg


@pytest.mark.parametrize("make", [
    lambda: _system_blocks(synth.grid_2d_four_lines(32))[0],
    lambda: _system_blocks(synth.regular_3d(n=10, seed=3))[0],
    lambda: _system_blocks(synth.regular_3d(n=10, seed=3))[1],
])
def test_tentative_orthonormal_and_coarse_symmetric(make):
    A = make()
    H = amg.setup(A, amg.AMGOptions(max_coarse=20))
    assert len(H.levels) >= 2
    for lv in H.levels[:-1]:
        Pt = amg.tentative(lv.agg, int(lv.agg.max()) + 1)
        G = (Pt.T @ Pt).toarray()
        assert np.allclose(G, np.eye(G.shape[0]), atol=1e-15)
        assert (lv.R != lv.P.T).nnz == 0
    for lv in H.levels[1:]:
        D = (lv.A - lv.A.T)
        assert abs(D).max() <= 1e-13 * abs(lv.A).max()


def test_near_nullspace_preserved_on_neumann_graph():
    """Pure-Neumann graph Laplacian (A 1 = 0): with every node aggregated,
    c_a = sqrt(|agg_a|) gives P_tent c = 1, hence P c = 1 and A_c c = 0."""
    m = 9
    A = _grid(m).tolil()
    for i in range(m * m):  # turn the Dirichlet-like grid into a pure-Neumann one
        A[i, i] = 0.0
        A[i, i] = -A[i].sum()
    A = sp.csr_matrix(A)
    assert np.allclose(A @ np.ones(m * m), 0.0)
    agg, n_agg = amg.aggregate(amg.strong_neighbours(A, 0.08))
    assert np.all(agg >= 0)
    c = np.sqrt(np.bincount(agg).astype(float))
    Pt = amg.tentative(agg, n_agg)
    P = amg.smoothed_prolongator(A, Pt)
    assert np.allclose(Pt @ c, 1.0, atol=1e-14)
    assert np.allclose(P @ c, 1.0, atol=1e-13)
    Ac = P.T @ A @ P
    assert np.allclose(Ac @ c, 0.0, atol=1e-12)


def test_one_level_hierarchy_is_exact_solve():
    S, Agg = _system_blocks(synth.tiny_2d(10))
    H = amg.setup(S)
    assert len(H.levels) == 1 and H.coarse_dense is not None
    b = synth.random_vector(S.shape[0], 1)
    x = amg.vcycle(H, b)
    assert np.allclose(S @ x, b, rtol=0, atol=1e-12 * np.linalg.norm(b))


def _operator(H, n):
    return np.column_stack([amg.vcycle(H, e) for e in np.eye(n)])


def test_two_level_cycle_is_textbook_two_grid():
    """I - B A = (I - D^-1 A)(I - P A_c^-1 R A)(I - D^-1 A), with D the l1
    diagonal, for a two-level hierarchy with an exact coarse solve."""
    S, _ = _system_blocks(synth.grid_2d_four_lines(24))
    n = S.shape[0]
    H = amg.setup(S, amg.AMGOptions(max_levels=2))
    assert len(H.levels) == 2 and H.coarse_dense is not None
    A = S.toarray()
    lv = H.levels[0]
    P, R = lv.P.toarray(), lv.R.toarray()
    Ac = H.levels[1].A.toarray()
    I = np.eye(n)
    Sm = I - A / lv.d_l1[:, None]
    E = Sm @ (I - P @ np.linalg.solve(Ac, R @ A)) @ Sm
    B = _operator(H, n)
    assert np.allclose(I - B @ A, E, atol=1e-10)


def test_vcycle_operator_symmetric_positive_definite():
    S, _ = _system_blocks(synth.tiny_3d(6, seed=2))
    n = S.shape[0]
    H = amg.setup(S, amg.AMGOptions(max_coarse=10))
    assert len(H.levels) >= 3
    B = _operator(H, n)
    assert np.allclose(B, B.T, atol=1e-12 * np.abs(B).max())
    assert np.linalg.eigvalsh(0.5 * (B + B.T)).min() > 0.0


def test_coarsest_without_dense_uses_l1_jacobi():
    S, _ = _system_blocks(synth.tiny_2d(12))
    H = amg.setup(S, amg.AMGOptions(max_dense=10, max_levels=1))
    assert H.coarse_dense is None
    b = synth.random_vector(S.shape[0], 4)
    x = amg.vcycle(H, b)
    d = H.levels[0].d_l1
    y = b / d
    for _ in range(3):
        y = y + (b - S @ y) / d
    assert np.array_equal(x, y)


def test_stopping_rules():
    S, _ = _system_blocks(synth.regular_3d(n=12, seed=1))
    H = amg.setup(S)
    sizes = H.sizes()
    assert sizes[-1] <= 400 or len(sizes) == 10
    assert all(sizes[i + 1] <= 0.9 * sizes[i] for i in range(len(sizes) - 1))
    assert all(s > 400 for s in sizes[:-1])


def test_smoothed_prolongator_closed_form_chain():
    """Chain of 7 with aggregates {0,1}, {2,3,4}, {5,6}: D = diag(A) =
    (1,2,2,2,2,2,1), Gershgorin rho = 2, omega = 2/3.  Expanding
    P = P_tent - omega D^-1 A P_tent by hand gives the columns below."""
    A = _chain(7)
    agg, n_agg = amg.aggregate(amg.strong_neighbours(A, 0.08))
    P = amg.smoothed_prolongator(A, amg.tentative(agg, n_agg)).toarray()
    s2, s3 = np.sqrt(2.0), np.sqrt(3.0)
    expect = np.zeros((7, 3))
    expect[:3, 0] = [1 / s2, 2 / (3 * s2), 1 / (3 * s2)]
    expect[1:6, 1] = [1 / (3 * s3), 2 / (3 * s3), 1 / s3, 2 / (3 * s3), 1 / (3 * s3)]
    expect[4:, 2] = [1 / (3 * s2), 2 / (3 * s2), 1 / s2]
    assert np.allclose(P, expect, rtol=0, atol=1e-15)


def test_l1_diagonal_definition():
    A = sp.csr_matrix(np.array([[4.0, -1.5, 0.0], [-1.5, 3.0, 2.0], [0.0, 2.0, -5.0]]))
    assert np.array_equal(amg.l1_diagonal(A), [5.5, 6.5, 7.0])


def _recursion_operator(H, lvl, pre, post, sweeps):
    """B_l of the textbook multigrid recursion (operator algebra, not the
    oracle's update sequence): B_L = A_L^-1 (dense coarsest) or
    (I - S_L^sweeps) A_L^-1 (swept coarsest); for l < L,
    I - B_l A_l = S_l^post (I - P_l B_{l+1} R_l A_l) S_l^pre, S_l = I - D_l^-1 A_l."""
    lv = H.levels[lvl]
    A = lv.A.toarray()
    n = A.shape[0]
    I = np.eye(n)
    Ainv = np.linalg.inv(A)
    S = I - A / lv.d_l1[:, None]
    if lvl == len(H.levels) - 1:
        if H.coarse_dense is not None:
            return Ainv
        return (I - np.linalg.matrix_power(S, sweeps)) @ Ainv
    Bc = _recursion_operator(H, lvl + 1, pre, post, sweeps)
    P, R = lv.P.toarray(), lv.R.toarray()
    E = np.linalg.matrix_power(S, post) @ (I - P @ Bc @ R @ A) @ np.linalg.matrix_power(S, pre)
    return (I - E) @ Ainv


@pytest.mark.parametrize("pre,post", [(1, 1), (2, 1), (1, 3), (2, 2)])
@pytest.mark.parametrize("dense", [True, False])
def test_vcycle_equals_multigrid_recursion(pre, post, dense):
    """A V-cycle over three or more levels, with the given sweep counts and a
    dense or swept (four l1-Jacobi sweeps) coarsest level, applies exactly the
    operator of the textbook recursion."""
    S, _ = _system_blocks(synth.tiny_3d(6, seed=2))
    n = S.shape[0]
    opts = amg.AMGOptions(max_coarse=10, max_dense=2000 if dense else 2, pre_sweeps=pre, post_sweeps=post)
    H = amg.setup(S, opts)
    assert len(H.levels) >= 3 and (H.coarse_dense is not None) == dense
    B = _recursion_operator(H, 0, pre, post, opts.coarse_sweeps)
    V = _operator(H, n)
    assert np.allclose(V, B, rtol=0, atol=1e-10 * np.abs(B).max())


@pytest.mark.parametrize("k", [1, 2, 4, 7])
def test_l1_jacobi_sweeps_closed_form(k):
    """k undamped l1-Jacobi sweeps from zero are the truncated Neumann series
    of A^-1 in the smoothing matrix: x_k = (I - (I - D^-1 A)^k) A^-1 b.  The
    coarsest level without a dense inverse runs coarse_sweeps of them."""
    S, _ = _system_blocks(synth.tiny_2d(12))
    H = amg.setup(S, amg.AMGOptions(max_dense=10, max_levels=1, coarse_sweeps=k))
    assert H.coarse_dense is None and len(H.levels) == 1
    A = S.toarray()
    d = H.levels[0].d_l1
    b = synth.random_vector(S.shape[0], 4)
    G = np.eye(A.shape[0]) - A / d[:, None]
    expect = (np.eye(A.shape[0]) - np.linalg.matrix_power(G, k)) @ np.linalg.solve(A, b)
    x = amg.vcycle(H, b)
    assert np.allclose(x, expect, rtol=0, atol=1e-12 * np.abs(expect).max())


@pytest.mark.parametrize("cycles", [2, 3])
@pytest.mark.parametrize("dense", [True, False])
def test_cycles_closed_form(cycles, dense):
    """nu V-cycles as a stationary iteration from zero: the error after nu
    steps is E^nu times the initial error, so x_nu = (I - E^nu) A^-1 b with
    E = I - B A and B the recursion operator (independent of the oracle's
    update sequence)."""
    S, _ = _system_blocks(synth.tiny_3d(6, seed=2))
    n = S.shape[0]
    opts = amg.AMGOptions(max_coarse=10, max_dense=2000 if dense else 2)
    H = amg.setup(S, opts)
    A = S.toarray()
    B = _recursion_operator(H, 0, 1, 1, opts.coarse_sweeps)
    E = np.eye(n) - B @ A
    b = synth.random_vector(n, 9)
    expect = (np.eye(n) - np.linalg.matrix_power(E, cycles)) @ np.linalg.solve(A, b)
    x = amg.apply_cycles(H, b, cycles)
    assert np.allclose(x, expect, rtol=0, atol=1e-10 * np.abs(expect).max())


@pytest.mark.parametrize("make,expect", [
    (lambda: _chain(7), [0, 1, 0, 1, 0, 1, 0]),
    (_pass2_graph, [0, 1, 0, 0, 1, 2]),  # edges 0-1, 1-2, 2-5, 3-4, 4-5, worked by hand in natural order
    (lambda: _grid(4), [(i + j) % 2 for j in range(4) for i in range(4)]),  # red-black
])
def test_greedy_colours_by_hand(make, expect):
    assert np.array_equal(amg.greedy_colours(make()), expect)


def _gs_dense(A, colour):
    """Forward / backward multicolour Gauss-Seidel as dense triangular
    operators in the (colour, index) order: x -> (D+L)^-1 (b - U x) and
    x -> (D+U)^-1 (b - L x), mapped back to the natural order."""
    import scipy.linalg as la
    n = A.shape[0]
    P = np.lexsort((np.arange(n), colour))  # rows sorted by colour, then index
    Ap = A[np.ix_(P, P)]
    Lo, Up = np.tril(Ap), np.triu(Ap)

    def fwd(b, x):
        y = la.solve_triangular(Lo, b[P] - np.triu(Ap, 1) @ x[P], lower=True)
        out = np.empty(n)
        out[P] = y
        return out

    def bwd(b, x):
        y = la.solve_triangular(Up, b[P] - np.tril(Ap, -1) @ x[P], lower=False)
        out = np.empty(n)
        out[P] = y
        return out
    return fwd, bwd


@pytest.mark.parametrize("make", [lambda: _system_blocks(synth.tiny_3d(6, seed=2))[0],
                                  lambda: _system_blocks(synth.random_2d(3, n_range=(12, 16)))[0]])
def test_multicolour_sweep_is_gauss_seidel_in_colour_order(make):
    """A valid colouring (no two coupled nodes share a colour); one forward
    and one backward sweep equal the dense triangular solves of
    Gauss-Seidel in the (colour, index) order."""
    S = sp.csr_matrix(make())
    col = amg.greedy_colours(S)
    G = (abs(S) + abs(S.T)).tocoo()
    assert all(col[i] != col[j] for i, j in zip(G.row, G.col) if i != j)
    A = S.toarray()
    fwd, bwd = _gs_dense(A, col)
    b = synth.random_vector(S.shape[0], 12)
    x0 = synth.random_vector(S.shape[0], 13)
    scale = np.abs(fwd(b, x0)).max()
    assert np.allclose(amg.gs_sweep(S, b, x0, col, True), fwd(b, x0), rtol=0, atol=1e-12 * scale)
    assert np.allclose(amg.gs_sweep(S, b, x0, col, False), bwd(b, x0), rtol=0, atol=1e-12 * scale)


def _gs_recursion_operator(H, lvl, pre, post):
    lv = H.levels[lvl]
    A = lv.A.toarray()
    n = A.shape[0]
    I = np.eye(n)
    Ainv = np.linalg.inv(A)
    if lvl == len(H.levels) - 1:
        return Ainv  # dense coarsest
    fwd, bwd = _gs_dense(A, lv.colour)
    # smoothing matrices I - M A with M the sweep's operator on b from x = 0
    Mf = np.column_stack([fwd(e, np.zeros(n)) for e in I])
    Mb = np.column_stack([bwd(e, np.zeros(n)) for e in I])
    Sf, Sb = I - Mf @ A, I - Mb @ A
    Bc = _gs_recursion_operator(H, lvl + 1, pre, post)
    P, R = lv.P.toarray(), lv.R.toarray()
    E = np.linalg.matrix_power(Sb, post) @ (I - P @ Bc @ R @ A) @ np.linalg.matrix_power(Sf, pre)
    return (I - E) @ Ainv


@pytest.mark.parametrize("pre,post", [(1, 1), (2, 1), (1, 2)])
def test_gauss_seidel_vcycle_equals_recursion_and_is_symmetric(pre, post):
    """With multicolour Gauss-Seidel (forward before, backward after) the
    V-cycle applies the textbook recursion's operator; with equal sweep
    counts it is symmetric, as the forward and backward sweeps are adjoint."""
    S, _ = _system_blocks(synth.tiny_3d(6, seed=2))
    n = S.shape[0]
    H = amg.setup(S, amg.AMGOptions(max_coarse=10, smoother="gs", pre_sweeps=pre, post_sweeps=post))
    assert len(H.levels) >= 3 and H.coarse_dense is not None
    B = _gs_recursion_operator(H, 0, pre, post)
    V = _operator(H, n)
    assert np.allclose(V, B, rtol=0, atol=1e-10 * np.abs(B).max())
    if pre == post:
        assert np.allclose(V, V.T, rtol=0, atol=1e-10 * np.abs(V).max())


def test_dimension_aware_aggregation_by_hand():
    """Chain of 7 whose first three nodes carry one label and last four
    another (two subdomains of different dimension): the strength graph
    loses the edge 2-3, pass 1 makes {0,1}, {3,4}, {6,5}, pass 2 attaches 2
    to {0,1}: [0,0,0,1,1,2,2] (unlabelled: the golden chain aggregation)."""
    labels = np.array([0, 0, 0, 1, 1, 1, 1])
    agg, n_agg = amg.aggregate(amg.strong_neighbours(_chain(7), 0.08, labels))
    assert np.array_equal(agg, [0, 0, 0, 1, 1, 2, 2]) and n_agg == 3
    plain, _ = amg.aggregate(amg.strong_neighbours(_chain(7), 0.08))
    assert np.array_equal(plain, _golden("aggregation_chain7.txt"))


@pytest.mark.parametrize("make", [lambda: synth.grid_2d_four_lines(16), lambda: synth.tiny_3d(7, seed=1)])
def test_dimension_aware_aggregation_properties(make):
    """On the interface-flux system's S~ (host, fracture, line and point
    unknowns): no finest-level aggregate mixes dimensions, coarser levels may;
    with one label for all unknowns the hierarchy is the unlabelled one."""
    from oracle import mixed_dim as md, precond
    A, b, part, info = md.assemble_flux(make())
    lab = info["labels"]
    M = precond.ML(A, part, amg_opts=amg.AMGOptions(max_coarse=20), labels=lab)
    lo = lab[M.omega]
    agg = M.H_omega.levels[0].agg
    assert len(np.unique(lo)) >= 3
    for a in np.unique(agg[agg >= 0]):
        assert len(np.unique(lo[agg == a])) == 1
    M1 = precond.ML(A, part, amg_opts=amg.AMGOptions(max_coarse=20), labels=np.zeros_like(lab))
    M0 = precond.ML(A, part, amg_opts=amg.AMGOptions(max_coarse=20))
    assert M1.H_omega.sizes() == M0.H_omega.sizes()
    for l1, l0 in zip(M1.H_omega.levels, M0.H_omega.levels):
        assert (l1.A != l0.A).nnz == 0
