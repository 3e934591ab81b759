"""Oracle assembly: two-point flux discretisation of the mixed-dimensional
scalar elliptic model on a Cartesian grid.  TEST INFRASTRUCTURE ONLY.

Model (Section 2.1): in every subdomain the conservation law eq. (1) holds
with the interface fluxes as source terms; the interface flux follows the
Darcy-type law eq. (2) and enters the higher-dimensional neighbour as a
Neumann term eq. (3).  The paper discretises with MPFA on simplex meshes
(Section 2.2); here every subdomain uses two-point fluxes on a uniform grid,
which is the reading adopted for this library:

* host cells, size h = 1/n, face area A = h^(dim-1); a host cell's half
  transmissibility to a face is t = 2 K A / h and two host cells sharing an
  unfractured face couple with the harmonic combination t_L t_R/(t_L+t_R);
* a fracture cell sits on one host face.  Its tangential transmissibility is
  K_par * a (a = aperture); its normal coupling per unit area is kappa/(a/2).
  Host cell X and fracture cell f couple in series:
  T_Xf = 1 / (1/t_X + a/(2 kappa A)).  A fractured host face has no direct
  host-host coupling: the two sides meet only through f (eq. 3);
* fracture cells meet at facets (grid vertices in 2D, grid edges in 3D).
  A fracture cell's half transmissibility toward a facet of measure |e|
  (1 in 2D, h in 3D) is tau = 2 K_par a |e| / h.  At an interior facet with
  incident cells F (|F| >= 2) every pair couples with tau_f tau_g / sum(tau)
  (star-delta elimination of the facet unknown; for |F| = 2 this is the
  harmonic combination, so in-plane neighbours and intersections follow one
  rule).  A single incident cell at an interior facet is a no-flux tip
  (Figure 1 caption).  A facet on a Dirichlet boundary ties each incident
  cell to the boundary value through its own tau;
* Dirichlet host faces add t to the diagonal and t*g to the right-hand side;
  other boundaries are no-flux; host sources add f*h^dim.

Unknown order: host cells (x fastest), then fracture cells fracture by
fracture, first tangential axis fastest; ``part`` is 0 for host (Omega) and
1 for fracture (Gamma) unknowns (eq. 4).

Pins: manufactured linear pressure, 1D series-resistance closed form,
symmetry, M-matrix sign pattern, flux conservation and unknown/nonzero
counts (tests/test_oracle_assembly.py).
"""

from __future__ import annotations

import itertools
from collections import defaultdict

import numpy as np
import scipy.sparse as sp


def host_index(n: int, dim: int, coords) -> int:
    """Linear index of host cell with integer coordinates (x, y[, z])."""
    c = 0
    stride = 1
    for a in range(dim):
        c += coords[a] * stride
        stride *= n
    return c


def fracture_cells(sc):
    """List of (fracture_number, tangential_cell_coords) in unknown order,
    plus a dict from host face (axis, index, tangential coords) to the
    fracture cell number (0-based within the fracture block)."""
    cells = []
    face_to_cell = {}
    for fi, fr in enumerate(sc.fractures):
        ranges = [range(l, u) for l, u in zip(fr.lo, fr.hi)]
        # first tangential axis fastest -> iterate the last one outermost
        for tup in itertools.product(*reversed(ranges)):
            t = tuple(reversed(tup))
            key = (fr.axis, fr.index, t)
            if key in face_to_cell:
                raise ValueError("two fracture cells on one host face")
            face_to_cell[key] = len(cells)
            cells.append((fi, t))
    return cells, face_to_cell


def assemble(sc):
    """Return (A, b, part): A scipy CSR FP64, b FP64, part int32."""
    n, dim = sc.n, sc.dim
    h = 1.0 / n
    area = h ** (dim - 1)
    vol = h ** dim
    n_host = n ** dim
    cells, face_to_cell = fracture_cells(sc)
    n_tot = n_host + len(cells)

    diag = np.zeros(n_tot)
    rhs = np.zeros(n_tot)
    rows, cols, vals = [], [], []

    def couple(u, v, T):
        diag[u] += T
        diag[v] += T
        rows.extend((u, v))
        cols.extend((v, u))
        vals.extend((-T, -T))

    k = np.asarray(sc.k_host, dtype=np.float64)
    t_half = 2.0 * k * area / h  # host half transmissibility (all faces equal on a cube grid)

    # ---- host faces, one at a time -------------------------------------------------
    for axis in range(dim):
        tang = [a for a in range(dim) if a != axis]
        for tcoords in itertools.product(range(n), repeat=dim - 1):
            coords = [0] * dim
            for a, t in zip(tang, tcoords):
                coords[a] = t
            # boundary faces
            for side, q in ((0, 0), (1, n - 1)):
                g = sc.dirichlet.get((axis, side))
                if g is None:
                    continue
                coords[axis] = q
                c = host_index(n, dim, coords)
                diag[c] += t_half[c]
                rhs[c] += t_half[c] * g
            # interior faces
            for q in range(1, n):
                coords[axis] = q - 1
                cl = host_index(n, dim, coords)
                coords[axis] = q
                cr = host_index(n, dim, coords)
                f = face_to_cell.get((axis, q, tuple(tcoords)))
                if f is None:
                    tl, tr = t_half[cl], t_half[cr]
                    couple(cl, cr, tl * tr / (tl + tr))
                else:
                    fr = sc.fractures[cells[f][0]]
                    normal = fr.aperture / (2.0 * fr.kappa * area)
                    couple(cl, n_host + f, 1.0 / (1.0 / t_half[cl] + normal))
                    couple(n_host + f, cr, 1.0 / (1.0 / t_half[cr] + normal))

    # ---- fracture facets ---------------------------------------------------------------
    facet_measure = 1.0 if dim == 2 else h
    facets = defaultdict(list)  # key -> list of (cell number, tau)
    for f, (fi, t) in enumerate(cells):
        fr = sc.fractures[fi]
        tang = [a for a in range(dim) if a != fr.axis]
        tau = 2.0 * fr.k_par * fr.aperture * facet_measure / h
        for m, bm in enumerate(tang):
            for s in (0, 1):
                pt = [0] * dim
                pt[fr.axis] = fr.index
                pt[bm] = t[m] + s
                direction = -1
                for m2, b2 in enumerate(tang):
                    if b2 != bm:
                        pt[b2] = t[m2]
                        direction = b2
                facets[(direction, tuple(pt))].append((f, tau))

    for (direction, pt), inc in facets.items():
        bnd = None
        for a in range(dim):
            if a == direction:
                continue
            if pt[a] == 0:
                bnd = (a, 0)
            elif pt[a] == n:
                bnd = (a, 1)
        if bnd is not None:
            g = sc.dirichlet.get(bnd)
            if g is not None:
                for f, tau in inc:
                    diag[n_host + f] += tau
                    rhs[n_host + f] += tau * g
            continue
        if len(inc) < 2:
            continue  # no-flux tip
        tot = sum(tau for _, tau in inc)
        if tot == 0.0:
            continue  # no tangential conductivity at this facet
        for (f, tf), (g2, tg) in itertools.combinations(inc, 2):
            couple(n_host + f, n_host + g2, tf * tg / tot)

    if sc.source is not None:
        rhs[:n_host] += np.asarray(sc.source, dtype=np.float64) * vol

    rows.extend(range(n_tot))
    cols.extend(range(n_tot))
    vals.extend(diag.tolist())
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n_tot, n_tot)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    part = np.zeros(n_tot, dtype=np.int32)
    part[n_host:] = 1
    return A, rhs, part
