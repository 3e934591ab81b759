"""Pins of the oracle assembly (two-point flux reading of Section 2.1,
eqs. (1)-(3), giving the block system of eq. (4)) against closed forms and
structural facts that do not depend on the assembly code."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import Fracture, Scenario
from oracle import assembly as oa
from oracle import blocks as ob


def _dense_solve(A, b):
    return np.linalg.solve(A.toarray(), b)


def test_counts_2d_four_lines():
    A, b, part = oa.assemble(synth.grid_2d_four_lines(32))
    # 32x32 host cells + 4 lines x 32 fracture cells
    assert A.shape == (1152, 1152)
    assert int(part.sum()) == 128
    # host 5-point pattern minus 128 fractured faces (2 entries each), plus
    # 2 host neighbours per fracture cell in both off-diagonal blocks, plus
    # the fracture block: diagonal, 4*31 in-line pairs and 4 crossings with
    # 4 extra pairs each.
    host = 32 * 32 + 4 * 32 * 31
    expected = (host - 2 * 128) + 2 * (2 * 128) + (128 + 2 * (4 * 31 + 4 * 4))
    assert expected == 5656
    assert A.nnz == expected


@pytest.mark.parametrize("n", [4, 8, 12])
def test_counts_3d_nine_planes(n):
    A, b, part = oa.assemble(synth.regular_3d(n=n, sigma=1.0, seed=n))
    _, _, Aoo, Aog, Ago, Agg = ob.split(A, part)
    assert Aoo.shape[0] == n ** 3
    assert Agg.shape[0] == 9 * n * n
    seven_point = n ** 3 + 6 * n * n * (n - 1)
    assert Aoo.nnz == seven_point - 18 * n * n
    assert Aog.nnz == Ago.nnz == 18 * n * n
    # in-plane pairs 9 * 2n(n-1); 27 plane pairs meet along n edges each, with
    # 4 incident faces per edge = 4 cross-plane pairs per edge
    assert Agg.nnz == 9 * n * n + 2 * (18 * n * (n - 1) + 4 * 27 * n)


SCENARIOS = [
    lambda: synth.grid_2d_four_lines(16, 1e-4, 1e4),
    lambda: synth.tiny_2d(10, seed=3),
    lambda: synth.tiny_3d(6, seed=4),
    lambda: synth.regular_3d(n=8, k_par=1e-4, kappa=1e-4, seed=1),
    lambda: synth.random_2d(5, n_range=(16, 24), max_segments=8),
]


@pytest.mark.parametrize("make", SCENARIOS)
def test_symmetry_and_mmatrix(make):
    sc = make()
    A, b, part = oa.assemble(sc)
    # bitwise symmetric; A_OG = A_GO^T (Section 3.1)
    assert (A != A.T).nnz == 0
    _, _, _, Aog, Ago, _ = ob.split(A, part)
    assert (Aog != Ago.T).nnz == 0
    C = A.tocoo()
    off = C.row != C.col
    assert np.all(C.data[off] <= 0.0)
    assert np.all(A.diagonal() > 0.0)
    # row sums: zero away from Dirichlet contact, positive where a cell
    # (host or fracture) touches the x = 0 or x = 1 boundary
    rs = np.asarray(A.sum(axis=1)).ravel()
    touches = b != 0.0
    scale = np.abs(A.diagonal())
    assert np.all(rs >= -1e-13 * scale)
    # cells that touch the p = 1 boundary carry a nonzero rhs
    assert np.all(rs[touches] > 0.0)


@pytest.mark.parametrize("make", SCENARIOS)
def test_constant_pressure_is_reproduced(make):
    """With the same Dirichlet value on every Dirichlet face and no sources,
    p == g everywhere: no coupling may create or destroy mass."""
    sc = make()
    sc = Scenario(sc.dim, sc.n, sc.k_host, sc.fractures, {k: 0.7 for k in sc.dirichlet})
    A, b, part = oa.assemble(sc)
    p = _dense_solve(A, b)
    assert np.max(np.abs(p - 0.7)) < 1e-10


def _linear_scenario(dim):
    if dim == 2:
        n = 16
        fr = [Fracture(1, 4, (0,), (n,), 3e2, 5e-3, 1e-3),
              Fracture(1, 11, (0,), (n,), 1e-4, 1e4, 1e-4)]
    else:
        n = 8
        fr = [Fracture(1, 2, (0, 0), (n, n), 1e4, 1e4, 1e-4),
              Fracture(1, 5, (0, 0), (n, n), 1.0, 1e-4, 1e-4),
              Fracture(2, 3, (0, 0), (n, n), 20.0, 3.0, 1e-2)]
    return Scenario(dim, n, np.full(n ** dim, 2.5), fr, {(0, 0): 1.0, (0, 1): 0.0})


def _x_centres(sc):
    n, h = sc.n, 1.0 / sc.n
    idx = np.arange(sc.n_host)
    xs = [((idx % n) + 0.5) * h]
    for fr in sc.fractures:
        # x is the first tangential axis of planes normal to y or z
        t0 = np.arange(fr.lo[0], fr.hi[0])
        reps = fr.n_cells() // t0.size
        xs.append(np.tile((t0 + 0.5) * h, reps))
    return np.concatenate(xs)


@pytest.mark.parametrize("dim", [2, 3])
def test_manufactured_linear_pressure(dim):
    """p = 1 - x is exact for two-point flux with constant host permeability
    when every fracture is parallel to the gradient and spans the domain
    (host and fracture pressures coincide across the interface, so eq. (2)
    carries no flux, and intersections connect equal pressures)."""
    sc = _linear_scenario(dim)
    A, b, part = oa.assemble(sc)
    p = _dense_solve(A, b)
    exact = 1.0 - _x_centres(sc)
    assert np.max(np.abs(p - exact)) < 1e-12


@pytest.mark.parametrize("dim", [2, 3])
def test_series_resistance_closed_form(dim):
    """Fractures normal to the gradient spanning the domain, host
    permeability varying along x only: every x-column is a chain of
    resistors.  Host half cell 1/t, t = 2 K h^(dim-1) / h; a fractured face
    adds the normal resistance a / (kappa h^(dim-1)) of eq. (2), split in
    two halves around the fracture cell."""
    n = 12 if dim == 2 else 6
    h = 1.0 / n
    area = h ** (dim - 1)
    kx = np.exp(np.sin(np.arange(n) * 1.7))
    k_host = np.tile(kx, n ** (dim - 1))
    lo, hi = (0,) * (dim - 1), (n,) * (dim - 1)
    fr = [Fracture(0, 3, lo, hi, 7.0, 2e-2, 1e-3), Fracture(0, n - 2, lo, hi, 1e-4, 5.0, 1e-4)]
    sc = Scenario(dim, n, k_host, fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = oa.assemble(sc)
    p = _dense_solve(A, b)

    t = 2.0 * kx * area / h
    face_extra = {3: fr[0].aperture / (fr[0].kappa * area), n - 2: fr[1].aperture / (fr[1].kappa * area)}
    R = 1.0 / t[0] + 1.0 / t[n - 1]
    for q in range(1, n):
        R += 1.0 / t[q - 1] + 1.0 / t[q] + face_extra.get(q, 0.0)
    Q = 1.0 / R
    ph = np.zeros(n)
    ph[0] = 1.0 - Q / t[0]
    pf = {}
    for q in range(1, n):
        if q in face_extra:
            pf[q] = ph[q - 1] - Q * (1.0 / t[q - 1] + 0.5 * face_extra[q])
        ph[q] = ph[q - 1] - Q * (1.0 / t[q - 1] + 1.0 / t[q] + face_extra.get(q, 0.0))
    host = p[: n ** dim].reshape((n,) * dim)
    for col in np.ndindex(*(n,) * (dim - 1)):
        line = host[col] if dim == 2 else host[col[0], col[1], :]
        # host arrays are indexed [z][y][x]; the last axis is x
        assert np.allclose(line, ph, rtol=0, atol=1e-13)
    off = n ** dim
    m = n ** (dim - 1)
    assert np.allclose(p[off:off + m], pf[3], rtol=0, atol=1e-13)
    assert np.allclose(p[off + m:off + 2 * m], pf[n - 2], rtol=0, atol=1e-13)
    # the outflow through x = 1 equals the closed-form flow per column
    assert abs(t[n - 1] * ph[n - 1] - Q) < 1e-13 * Q + 1e-15


def test_sources_scale_with_cell_volume():
    """A uniform source f on a closed-except-Dirichlet domain: the total
    Dirichlet outflow equals f times the domain measure (global balance of
    eq. (1) summed over all cells)."""
    sc = synth.tiny_2d(12, seed=2)
    sc = Scenario(2, sc.n, sc.k_host, sc.fractures, {(0, 0): 0.0, (0, 1): 0.0},
                  source=np.full(sc.n_host, 3.0))
    A, b, part = oa.assemble(sc)
    p = _dense_solve(A, b)
    # row sums of A are the Dirichlet transmissibilities; the outflow of a
    # row is rowsum * (p - 0)
    rs = np.asarray(A.sum(axis=1)).ravel()
    outflow = float(rs @ p)
    assert abs(outflow - 3.0) < 1e-10


def test_fracture_overlap_rejected():
    sc = Scenario(2, 8, np.ones(64), [Fracture(0, 4, (0,), (5,), 1, 1, 1e-2),
                                      Fracture(0, 4, (3,), (8,), 1, 1, 1e-2)],
                  {(0, 0): 1.0, (0, 1): 0.0})
    with pytest.raises(ValueError):
        oa.assemble(sc)


def test_unknown_order_fracture_cells():
    """Fracture cells follow host cells, fracture by fracture, first
    tangential axis fastest: check via the coupling pattern of a 3D plane."""
    n = 4
    fr = [Fracture(0, 2, (0, 1), (n, 3), 1.0, 1.0, 1e-2)]  # tangential (y, z): y in [0,4), z in [1,3)
    sc = Scenario(3, n, np.ones(n ** 3), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = oa.assemble(sc)
    off = n ** 3
    for f in range(8):
        y, z = f % 4, 1 + f // 4
        left = 1 + n * y + n * n * z  # host cell (x=1, y, z)
        right = 2 + n * y + n * n * z
        row = A.getrow(off + f)
        assert row[0, left] < 0 and row[0, right] < 0


@pytest.mark.parametrize("arms", ["cross", "tee"])
def test_star_delta_junction_closed_form(arms):
    """A full line y = 1/2 from the p = 1 to the p = 0 boundary, crossed at
    x = q h by a second line that ends in no-flux tips (both directions for a
    cross, one for a tee).  With the host decoupled (vanishing normal
    permeability) the hanging line carries no flux, so eliminating the
    junction must leave the through-line exactly linear, p = 1 - x, and give
    every hanging cell the junction pressure 1 - q h.  A per-pair harmonic
    rule would instead shorten the path across the junction."""
    n, q = 16, 4
    h = 1.0 / n
    tiny = 1e-30
    lo, hi = (1,), (n - 1,)
    if arms == "tee":
        lo = (n // 2,)
    fr = [Fracture(1, n // 2, (0,), (n,), 5.0, tiny, 1e-2),
          Fracture(0, q, lo, hi, 5.0, tiny, 1e-2)]
    sc = Scenario(2, n, np.ones(n * n), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part = oa.assemble(sc)
    p = _dense_solve(A, b)
    off = n * n
    through = p[off:off + n]
    assert np.allclose(through, 1.0 - (np.arange(n) + 0.5) * h, atol=1e-12)
    hanging = p[off + n:]
    assert np.allclose(hanging, 1.0 - q * h, atol=1e-12)
