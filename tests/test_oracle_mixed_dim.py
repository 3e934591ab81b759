"""Pins of the oracle mixed-dimensional assembly with interface fluxes
(the paper's own block reading of eq. (4): Omega = subdomain pressures,
Gamma = interface fluxes; Section 2.1 eqs. (1)-(3))."""

import numpy as np
import pytest
import scipy.sparse as sp

import synth
from synth import Fracture, Scenario
from oracle import assembly as oa
from oracle import mixed_dim as md
from oracle import solve as osv


def _blocks(A, part):
    A = sp.csr_matrix(A)
    o, g = np.flatnonzero(part == 0), np.flatnonzero(part == 1)
    return (A[o][:, o], A[o][:, g], A[g][:, o], A[g][:, g])


def _schur(A, part):
    Aoo, Aog, Ago, Agg = _blocks(A, part)
    return (Aoo - Aog @ sp.diags(1.0 / Agg.diagonal()) @ Ago).toarray()


def _x_planes(n, axes_q, k_par=7.0, kappa=3.0, aperture=1e-2):
    return [Fracture(ax, q, (0, 0), (n, n), k_par * (1 + ax), kappa * (2 - 0.5 * ax), aperture)
            for ax, q in axes_q]


@pytest.mark.parametrize("dim", [2, 3])
def test_linear_pressure_exact_with_planes_parallel_to_the_gradient(dim):
    """Constant host permeability, Dirichlet 1/0 on x, full fractures normal
    to y (and z): p = 1 - x in every host, fracture and line cell, and no
    flux crosses any interface (both sides have the same x)."""
    n = 8
    if dim == 2:
        fr = [Fracture(1, q, (0,), (n,), 5.0 * q, 0.7 * q, 1e-2) for q in (2, 5)]
    else:
        fr = _x_planes(n, [(1, 2), (1, 5), (2, 3), (2, 6)])
    sc = Scenario(dim, n, np.ones(n ** dim), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part, info = md.assemble_flux(sc)
    if dim == 3:
        assert info["intersection"] == 4 * n and info["point"] == 0  # x-lines, no points
    x = np.linalg.solve(A.toarray(), b)
    nc = info["cells"]
    assert np.abs(x[:nc] - (1.0 - info["centres"][:, 0])).max() <= 1e-12
    assert np.abs(x[nc:]).max() <= 1e-12


def test_series_closed_form_for_the_interface_fluxes():
    """Full fractures normal to the gradient, host permeability constant along
    y (a 1D problem per host row): every host-fracture interface carries the
    row flux Q = 1 / sum R (R = 1/t per Dirichlet half cell, 1/t_L + 1/t_R per
    plain face, 1/T_Lf + 1/T_fR per fractured face with
    1/T_Xf = 1/t_X + a/(2 kappa A)), positive on the low side and negative on
    the high side, and p_f = p_L - Q / T_Lf."""
    n = 10
    qs = [(3, 2.0, 0.3), (7, 0.5, 40.0)]  # (face index, k_par, kappa)
    a = 1e-3
    fr = [Fracture(0, q, (0,), (n,), kp, ka, a) for q, kp, ka in qs]
    kx = 1.0 + np.arange(n) * 0.37
    k = np.tile(kx, n)  # x fastest: constant along y
    sc = Scenario(2, n, k, fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part, info = md.assemble_flux(sc)
    x = np.linalg.solve(A.toarray(), b)
    h = 1.0 / n
    t = 2.0 * kx * h / h  # A = h in 2D
    R = 1.0 / t[0] + 1.0 / t[-1]
    Tl = {}
    for i in range(1, n):
        frq = [(kp, ka) for q, kp, ka in qs if q == i]
        if frq:
            kp, ka = frq[0]
            TL = 1.0 / (1.0 / t[i - 1] + a / (2.0 * ka * h))
            TR = 1.0 / (1.0 / t[i] + a / (2.0 * ka * h))
            R += 1.0 / TL + 1.0 / TR
            Tl[i] = TL
        else:
            R += 1.0 / t[i - 1] + 1.0 / t[i]
    Q = 1.0 / R
    nc = info["cells"]
    lam = x[nc:nc + 2 * info["fracture"]].reshape(-1, 2)  # (low side, high side) per fracture cell
    assert np.allclose(lam[:, 0], Q, rtol=1e-12) and np.allclose(lam[:, 1], -Q, rtol=1e-12)
    for f in range(info["fracture"]):
        q = qs[f // n][0]
        row = f % n
        pL = x[row * n + q - 1]
        assert abs(x[info["host"] + f] - (pL - Q / Tl[q])) <= 1e-12


@pytest.mark.parametrize("make", [lambda: synth.grid_2d_four_lines(12), lambda: synth.tiny_2d(8),
                                  lambda: synth.tiny_3d(6), lambda: synth.regular_3d(n=8, seed=1),
                                  lambda: synth.random_2d(4, n_range=(20, 30)),
                                  lambda: synth.random_3d(3, n_range=(8, 10))])
def test_block_structure_and_schur_complement(make):
    """A_GG diagonal and positive, A_GO = -A_OG^T, and the Schur complement
    S = A_OO - A_OG A_GG^-1 A_GO (which eq. (7) reproduces exactly, A_GG being
    diagonal) symmetric with non-positive off-diagonals and non-negative row
    sums, positive on Dirichlet-tied rows."""
    sc = make()
    A, b, part, info = md.assemble_flux(sc)
    Aoo, Aog, Ago, Agg = _blocks(A, part)
    assert (Agg - sp.diags(Agg.diagonal())).nnz == 0 and Agg.diagonal().min() > 0
    assert abs(Ago + Aog.T).max() == 0
    S = _schur(A, part)
    off = S - np.diag(np.diag(S))
    assert np.allclose(S, S.T, rtol=0, atol=1e-12 * np.abs(S).max())
    assert off.max() <= 0.0
    assert S.sum(axis=1).min() >= -1e-10 * np.abs(S).max()


def _cube_with_points(n=8, seed=5):
    """Two full planes normal to x; one plane normal to y and one normal to z
    that stop short of x = 0 and x = 1: lines in all three directions and two
    points, none touching the Dirichlet faces."""
    fr = [Fracture(0, 2, (0, 0), (n, n), 3.0, 2.0, 1e-2), Fracture(0, 5, (0, 0), (n, n), 0.5, 9.0, 1e-2),
          Fracture(1, 4, (1, 0), (n - 1, n), 4.0, 0.7, 1e-2), Fracture(2, 3, (1, 0), (n - 1, n), 1.5, 3.0, 1e-2)]
    k = np.exp(0.5 * np.random.default_rng(seed).standard_normal(n ** 3))
    return Scenario(3, n, k, fr, {(0, 0): 1.0, (0, 1): 0.0})


@pytest.mark.parametrize("make", [lambda: synth.tiny_2d(8), _cube_with_points])
def test_global_flux_conservation(make):
    """No sources: the flux entering at x = 0 equals the flux leaving at
    x = 1, counted over every Dirichlet-tied host cell from the host
    half transmissibility t = 2 K A / h.  An interface entered with a wrong
    sign in a cell row would create or destroy mass and break it.  (The
    fractures of these cases do not reach x = 0 or x = 1.)"""
    sc = make()
    for f in sc.fractures:
        assert f.axis == 0 or (f.lo[0] > 0 and f.hi[0] < sc.n)
    A, b, part, info = md.assemble_flux(sc)
    x = np.linalg.solve(A.toarray(), b)
    n, dim = sc.n, sc.dim
    h = 1.0 / n
    t = 2.0 * np.asarray(sc.k_host) * h ** (dim - 1) / h
    idx = np.arange(n ** dim)
    xi = idx % n
    fin = np.sum(t[xi == 0] * (1.0 - x[idx[xi == 0]]))
    fout = np.sum(t[xi == n - 1] * (x[idx[xi == n - 1]] - 0.0))
    assert fin > 0 and abs(fin - fout) <= 1e-10 * fin


def test_nine_plane_counts():
    """Nine full planes at (n/4, n/2, 3n/4) per axis: 27 lines of n cells, 27
    points, interfaces 2*9n^2 (host-fracture) + 4*27n (fracture-line) + 6*27
    (line-point)."""
    n = 8
    A, b, part, info = md.assemble_flux(synth.regular_3d(n=n, seed=0))
    assert info["fracture"] == 9 * n * n and info["intersection"] == 27 * n and info["point"] == 27
    assert info["interface"] == 18 * n * n + 108 * n + 162
    assert A.shape[0] == n ** 3 + info["fracture"] + 27 * n + 27 + info["interface"]
    assert int((part == 1).sum()) == info["interface"]


def _cube_with_lines_only(n=7):
    """Planes normal to x and y only (one partial, ending inside the cube):
    line cells along z, crossings and T-junctions, no points."""
    fr = [Fracture(0, 3, (0, 0), (n, n), 2.0, 5.0, 1e-2), Fracture(1, 2, (0, 0), (n, n), 0.7, 1.5, 1e-2),
          Fracture(1, 5, (1, 1), (6, n), 9.0, 0.2, 1e-2)]
    k = np.exp(0.5 * np.random.default_rng(8).standard_normal(n ** 3))
    return Scenario(3, n, k, fr, {(0, 0): 1.0, (0, 1): 0.0})


def _eliminate(S, keep):
    drop = np.setdiff1d(np.arange(S.shape[0]), keep)
    return S[np.ix_(keep, keep)] - S[np.ix_(keep, drop)] @ np.linalg.solve(S[np.ix_(drop, drop)],
                                                                           S[np.ix_(drop, keep)])


@pytest.mark.parametrize("make", [lambda: synth.grid_2d_four_lines(12), lambda: synth.tiny_2d(8, seed=3),
                                  lambda: synth.random_2d(6, n_range=(16, 24)),
                                  lambda: _cube_with_lines_only()])
def test_perfect_intersections_reduce_to_the_primal_star_delta_assembly(make):
    """With no normal resistance at intersections (and, in 3D, no conduction
    along line cells), eliminating the interface fluxes and the intersection
    pressures leaves exactly the primal assembly of the same scenario, whose
    facet rule is the star-delta elimination of the facet unknown: two
    independently written assemblies agree on every host-host, host-fracture
    and fracture-fracture coupling, Dirichlet ties and right-hand side."""
    sc = make()
    A, b, part, info = md.assemble_flux(sc, int_kappa_inf=True, line_k=0.0)
    assert info["point"] == 0 and info["intersection"] > 0
    S = _schur(A, part)
    nc = info["cells"]
    keep = np.arange(info["host"] + info["fracture"])
    S2 = _eliminate(S, keep)
    P, bp, pp = oa.assemble(sc)
    assert np.allclose(S2, P.toarray(), rtol=0, atol=1e-10 * np.abs(S2).max())
    assert np.allclose(b[:len(keep)], bp, rtol=0, atol=1e-14)
    assert np.allclose(b[len(keep):nc], 0.0)


def test_point_cells_star_delta_with_perfect_interfaces():
    """A 3D point cell with perfect interfaces couples its incident line
    cells i, j with tau_i tau_j / sum(tau) once eliminated (its row has no
    tangential part)."""
    n = 8
    sc = synth.regular_3d(n=n, seed=0, sigma=0.0, k_par=2.0, kappa=5.0, aperture=1e-2,
                          planes=[(0, 4), (1, 4), (2, 4)])
    A, b, part, info = md.assemble_flux(sc, int_kappa_inf=True)
    assert info["point"] == 1
    S = _schur(A, part)
    nc = info["cells"]
    pnt = nc - 1
    lines = np.flatnonzero(S[pnt, :nc] < 0)
    assert len(lines) == 6
    keep = np.setdiff1d(np.arange(nc), [pnt])
    S2 = _eliminate(S, keep)
    tau = 2.0 * 2.0 * 1e-2 ** 2 / (1.0 / n)
    li = [int(np.flatnonzero(keep == l)[0]) for l in lines]
    expect = tau * tau / (6 * tau)
    for a in li:
        for c in li:
            if a != c:
                extra = S2[a, c] - S[keep[a], keep[c]]
                assert abs(extra + expect) <= 1e-10 * expect


@pytest.mark.parametrize("make", [lambda: synth.grid_2d_four_lines(16), lambda: synth.tiny_3d(6, seed=2)])
def test_oracle_solve_on_the_flux_system(make):
    """The oracle's FGMRES with M_L (Gamma = the interface fluxes) reaches
    the dense solution of the nonsymmetric system."""
    sc = make()
    A, b, part, info = md.assemble_flux(sc)
    res, _, _ = osv.solve(A, b, part, osv.SolveOptions(tol=1e-12))
    xd = np.linalg.solve(A.toarray(), b)
    assert res.converged and np.linalg.norm(res.x - xd) <= 1e-9 * np.linalg.norm(xd)


def test_series_chain_through_intersection_points_2d():
    """A nearly insulating host (K = 1e-12) and three fractures forming the
    only path from x = 0 to x = 1: A along x from x = 0 to the point (m, q),
    B along y from (m, q) to (m, q2), C along x from (m, q2) to x = 1.  The
    flux is the series closed form Q = 1 / sum R with R = 1/tau for the
    Dirichlet half cells at both ends, 2/tau per face between two cells of
    one fracture, and 1/tau + 1/(2 kappa) (|e| = 1) for each
    fracture-point interface; every interface on the path carries Q,
    positive from A into the first point, negative from B into it, and so
    on."""
    n, m, q, q2 = 12, 5, 3, 8
    a = 1e-2
    A_, B_, C_ = (2.0, 0.8), (0.5, 3.0), (4.0, 0.3)  # (k_par, kappa)
    fr = [Fracture(1, q, (0,), (m,), A_[0], A_[1], a), Fracture(0, m, (q,), (q2,), B_[0], B_[1], a),
          Fracture(1, q2, (m,), (n,), C_[0], C_[1], a)]
    sc = Scenario(2, n, np.full(n * n, 1e-12), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part, info = md.assemble_flux(sc)
    assert info["intersection"] == 2
    h = 1.0 / n
    tau = [2.0 * k * a / h for k, _ in (A_, B_, C_)]
    lens = [m, q2 - q, n - m]
    R = 1.0 / tau[0] + 1.0 / tau[2]
    for t, L in zip(tau, lens):
        R += (L - 1) * 2.0 / t
    R += (1.0 / tau[0] + 1.0 / (2.0 * A_[1])) + 2 * (1.0 / tau[1] + 1.0 / (2.0 * B_[1])) + \
        (1.0 / tau[2] + 1.0 / (2.0 * C_[1]))
    Q = 1.0 / R
    x = np.linalg.solve(A.toarray(), b)
    nc = info["cells"]
    lam = x[nc + 2 * info["fracture"]:]  # fracture-point interfaces: point 1 (A, B), point 2 (B, C)
    assert len(lam) == 4
    assert np.allclose(lam, [Q, -Q, Q, -Q], rtol=1e-7)


def test_series_chain_through_a_point_3d():
    """Nearly insulating host and planes (K = 1e-12), lines made conducting
    (line_k = 1): the line along x at (y, z) = (q, q) from x = 0 to x = 1 is
    the only path; a small plane normal to x at x = m crosses it and makes a
    point there with four dead-end lines.  Q = 1 / sum R with R = 1/tau at
    both ends, 2/tau per face between line cells, and 1/tau + 1/(2 kappa a)
    for each line-point interface (tau = 2 a^2 / h, kappa the line's mean);
    the two through interfaces carry +Q and -Q, the dead ends nothing."""
    n, m, q = 10, 4, 5
    a = 0.05
    kap_y, kap_z, kap_x = 2.0, 6.0, 1.0
    fr = [Fracture(1, q, (0, q - 1), (n, q + 1), 1e-12, kap_y, a),
          Fracture(2, q, (0, q - 1), (n, q + 1), 1e-12, kap_z, a),
          Fracture(0, m, (q - 1, q - 1), (q + 1, q + 1), 1e-12, kap_x, a)]
    sc = Scenario(3, n, np.full(n ** 3, 1e-12), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part, info = md.assemble_flux(sc, line_k=1.0)
    assert info["point"] == 1
    h = 1.0 / n
    tau = 2.0 * a * a / h
    kap = 0.5 * (kap_y + kap_z)  # the x-line's incident planes
    R = 2.0 / tau + (n - 2) * 2.0 / tau + 2.0 * (1.0 / tau + 1.0 / (2.0 * kap * a))
    Q = 1.0 / R
    x = np.linalg.solve(A.toarray(), b)
    nc = info["cells"]
    ifc = info["interfaces"]
    pnt = nc - 1
    through = {}
    for e, (hi, lo) in enumerate(ifc):
        if lo == pnt:
            cen = info["centres"][hi]
            if abs(cen[1] - q * h) < 1e-12 and abs(cen[2] - q * h) < 1e-12:  # an x-line cell
                through[cen[0] < m * h] = x[nc + e]
            else:
                assert abs(x[nc + e]) <= 1e-7 * Q
    assert abs(through[True] - Q) <= 1e-7 * Q and abs(through[False] + Q) <= 1e-7 * Q


def test_series_chain_through_lines_3d():
    """The 2D chain extruded along z (no-flux z faces, so every z layer carries
    the same flux): fracture planes A, B, C meet along two lines of cells;
    with facet measure |e| = h each layer's flux is the 2D closed form with
    tau = 2 K_par a |e| / h and fracture-line interfaces 1/tau + 1/(2 kappa |e|)."""
    n, m, q, q2 = 8, 3, 2, 6
    a = 1e-2
    A_, B_, C_ = (2.0, 0.8), (0.5, 3.0), (4.0, 0.3)
    fr = [Fracture(1, q, (0, 0), (m, n), A_[0], A_[1], a), Fracture(0, m, (q, 0), (q2, n), B_[0], B_[1], a),
          Fracture(1, q2, (m, 0), (n, n), C_[0], C_[1], a)]
    sc = Scenario(3, n, np.full(n ** 3, 1e-12), fr, {(0, 0): 1.0, (0, 1): 0.0})
    A, b, part, info = md.assemble_flux(sc)
    assert info["intersection"] == 2 * n and info["point"] == 0
    h = 1.0 / n
    e = h
    tau = [2.0 * k * a * e / h for k, _ in (A_, B_, C_)]
    lens = [m, q2 - q, n - m]
    R = 1.0 / tau[0] + 1.0 / tau[2]
    for t, L in zip(tau, lens):
        R += (L - 1) * 2.0 / t
    R += (1.0 / tau[0] + 1.0 / (2.0 * A_[1] * e)) + 2 * (1.0 / tau[1] + 1.0 / (2.0 * B_[1] * e)) + \
        (1.0 / tau[2] + 1.0 / (2.0 * C_[1] * e))
    Q = 1.0 / R
    x = np.linalg.solve(A.toarray(), b)
    nc = info["cells"]
    lam = x[nc + 2 * info["fracture"]:]  # per line cell: its two incident fracture cells
    assert len(lam) == 4 * n
    assert np.allclose(np.abs(lam), Q, rtol=1e-7)
    assert np.isclose(lam.sum(), 0.0, atol=1e-7 * Q)
