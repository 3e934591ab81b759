"""Oracle assembly of the mixed-dimensional system in the paper's own block
reading: subdomain pressures and interface fluxes.  TEST INFRASTRUCTURE ONLY.

Section 2.1 splits the domain into subdomains of every dimension (the host,
fractures, and their intersection lines and points) joined by interfaces;
eq. (1) holds in every subdomain with the fluxes of the interfaces towards
its higher-dimensional neighbours as sources, eq. (2) gives each interface
flux from the pressure difference across it, and eq. (3) makes the same flux
a Neumann term of the higher-dimensional side.  Section 3.1 then orders the
unknowns as p_Omega (all subdomain pressures) and p_Gamma (all interface
fluxes), eq. (4).  Here every subdomain uses two-point fluxes on the uniform
grid (the discretisation reading of the primal assembly, `assembly.py`), and
intersections are explicit subdomains (in that module they are eliminated):

* subdomains: host cells (size h = 1/n, face area A = h^(dim-1)); fracture
  cells on host faces (aperture a); intersection cells on the grid facets
  where fracture cells of two or more planes meet (grid vertices in 2D:
  points; grid edges in 3D: line cells of length h); in 3D also point cells
  on the interior grid vertices where line cells of two or more directions
  meet.  An intersection cell takes the mean K_par, kappa and aperture of
  its incident cells;
* tangential two-point fluxes inside every subdomain: host faces t = 2 K A/h
  per side, harmonic across an unfractured face; fracture cells
  tau = 2 K_par a |e| / h toward a facet of measure |e| (1 in 2D, h in 3D),
  harmonic between the two coplanar cells of a facet that is not an
  intersection; line cells tau = 2 K_par a^2 / h toward each end, harmonic
  between two collinear line cells that meet at a vertex that is not a
  point.  A single cell at an interior facet is a no-flux tip (Figure 1
  caption); a facet or line end on a Dirichlet boundary ties the cell to the
  boundary value with its own half transmissibility;
* interfaces, one unknown Lambda (total flux, positive from the higher- to
  the lower-dimensional side) per (higher cell, lower cell) pair: host cell
  and fracture cell on its face, fracture cell and intersection cell at its
  facet, line cell and point at its end.  Its two-point law is eq. (2) in
  series with the higher cell's half transmissibility toward the interface:
  Lambda = T (p_high - p_low), 1/T = 1/t_high + w/(2 kappa m), where the
  lower subdomain's width w (the aperture) is crossed over half its width
  and m is the interface measure: host-fracture 1/T = 1/t_X + a/(2 kappa A);
  fracture-intersection 1/T = 1/tau_f + 1/(2 kappa |e|); line-point
  1/T = 1/tau_L + 1/(2 kappa a);
* rows: every cell row is eq. (1): tangential fluxes, plus Lambda for each
  interface where the cell is the higher side (eq. (3): an outflow), minus
  Lambda where it is the lower side, equal to the source; every interface
  row is eq. (2) divided by T: Lambda / T - p_high + p_low = 0.  So A_GG is
  diagonal and positive, A_GO = -A_OG^T (Section 3.1 does not rely on
  A_OG = A_GO^T), and S~ of eq. (7) equals the exact Schur complement.

Unknown order: host cells (x fastest); fracture cells (as `assembly.py`);
intersection cells by (direction, lower corner vertex, x fastest); points
by vertex; interfaces: host-fracture (fracture cell order, low side then
high side), fracture-intersection (intersection order, incident fracture
cells ascending), line-point (point order, incident line cells ascending).
``part`` is 0 for the pressures and 1 for the fluxes.

Options for the pins only: ``int_kappa_inf`` removes the normal resistance
of the interfaces at intersections (1/T = 1/tau); ``line_k`` replaces the
tangential permeability of every line cell (0: no conduction along lines).

Pins (tests/test_oracle_mixed_dim.py): exact linear pressure with planes
parallel to the gradient (line cells included); the 1D series closed form
for the host-fracture interface fluxes, and for chains of fractures (2D) or
line cells (3D) through intersection points, where the flux crosses the
intersection interfaces in series; A_GG diagonal positive, A_GO = -A_OG^T, and the
Schur complement symmetric with an M-matrix sign pattern; global flux
conservation; unknown counts of the nine-plane cube; with perfect
intersection interfaces (and no line conduction in 3D) the Schur complement
onto host and fracture cells equals the primal star-delta assembly.
"""

from __future__ import annotations

import itertools
from collections import defaultdict

import numpy as np
import scipy.sparse as sp

from .assembly import fracture_cells, host_index


def _vertex_index(n, dim, pt):
    c, stride = 0, 1
    for a in range(dim):
        c += pt[a] * stride
        stride *= n + 1
    return c


def _on_boundary(n, dim, pt, skip=None):
    """(axis, side) of a boundary face containing vertex set pt (ignoring
    axis `skip`), or None."""
    for a in range(dim):
        if a == skip:
            continue
        if pt[a] == 0:
            return (a, 0)
        if pt[a] == n:
            return (a, 1)
    return None


def assemble_flux(sc, int_kappa_inf=False, line_k=None):
    """Return (A, b, part, info): A scipy CSR FP64 (nonsymmetric), b FP64,
    part int32, info = counts of each kind of unknown."""
    n, dim = sc.n, sc.dim
    h = 1.0 / n
    area = h ** (dim - 1)
    n_host = n ** dim
    cells, face_to_cell = fracture_cells(sc)
    nf = len(cells)
    facet_measure = 1.0 if dim == 2 else h
    k = np.asarray(sc.k_host, dtype=np.float64)
    t_half = 2.0 * k * area / h

    # ---- facets of fracture cells ------------------------------------------------
    facets = defaultdict(list)  # (direction, lower corner) -> [(f, tau, plane)]
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
                facets[(direction, tuple(pt))].append((f, tau, (fr.axis, fr.index)))

    inter_keys = []  # interior facets where two or more planes meet, with some conduction
    plain = []       # other facets: (key, incident)
    for key, inc in facets.items():
        direction, pt = key
        interior = _on_boundary(n, dim, pt, skip=direction) is None
        planes = {p for _, _, p in inc}
        if interior and len(planes) >= 2 and sum(tau for _, tau, _ in inc) > 0.0:
            inter_keys.append(key)
        else:
            plain.append((key, inc))
    inter_keys.sort(key=lambda kd: (kd[0], _vertex_index(n, dim, kd[1])))
    ni = len(inter_keys)

    def inter_params(key):
        inc = facets[key]
        frs = [sc.fractures[cells[f][0]] for f, _, _ in inc]
        return (float(np.mean([fr.k_par for fr in frs])), float(np.mean([fr.kappa for fr in frs])),
                float(np.mean([fr.aperture for fr in frs])))

    # ---- points (3D): interior vertices where line cells of two or more directions meet
    ends = defaultdict(list)  # vertex -> [(line cell, direction)]
    if dim == 3:
        for i, (d, pt) in enumerate(inter_keys):
            for s in (0, 1):
                v = list(pt)
                v[d] += s
                ends[tuple(v)].append((i, d))
    point_keys = []
    for v, inc in ends.items():
        if _on_boundary(n, dim, v) is None and len({d for _, d in inc}) >= 2:
            point_keys.append(v)
    point_keys.sort(key=lambda v: _vertex_index(n, dim, v))
    npt = len(point_keys)

    # ---- unknown numbering -----------------------------------------------------------
    off_f = n_host
    off_i = off_f + nf
    off_p = off_i + ni
    n_cells = off_p + npt
    ifaces = []  # (high cell, low cell, 1/T)
    for f, (fi, t) in enumerate(cells):
        fr = sc.fractures[fi]
        tang = [a for a in range(dim) if a != fr.axis]
        normal = fr.aperture / (2.0 * fr.kappa * area)
        for side in (0, 1):
            coords = [0] * dim
            coords[fr.axis] = fr.index - 1 + side
            for a, tt in zip(tang, t):
                coords[a] = tt
            X = host_index(n, dim, coords)
            ifaces.append((X, off_f + f, 1.0 / t_half[X] + normal))
    for i, key in enumerate(inter_keys):
        for f, tau, _ in sorted(facets[key]):
            fr = sc.fractures[cells[f][0]]
            res = 1.0 / tau + (0.0 if int_kappa_inf else 1.0 / (2.0 * fr.kappa * facet_measure))
            ifaces.append((off_f + f, off_i + i, res))
    tau_line = {}
    for i, key in enumerate(inter_keys):
        kp, kap, ap = inter_params(key)
        if line_k is not None:
            kp = line_k
        tau_line[i] = 0.0 if dim == 2 else 2.0 * kp * ap * ap / h
    for p, v in enumerate(point_keys):
        for i, _ in sorted(ends[v]):
            kp, kap, ap = inter_params(inter_keys[i])
            if tau_line[i] == 0.0:
                raise ValueError("a point joins a line cell without tangential conduction")
            res = 1.0 / tau_line[i] + (0.0 if int_kappa_inf else 1.0 / (2.0 * kap * ap))
            ifaces.append((off_i + i, off_p + p, res))
    n_if = len(ifaces)
    n_tot = n_cells + n_if

    diag = np.zeros(n_tot)
    rhs = np.zeros(n_tot)
    rows, cols, vals = [], [], []

    def couple(u, v, T):
        diag[u] += T
        diag[v] += T
        rows.extend((u, v))
        cols.extend((v, u))
        vals.extend((-T, -T))

    # ---- host faces ----------------------------------------------------------------
    for axis in range(dim):
        tang = [a for a in range(dim) if a != axis]
        for tcoords in itertools.product(range(n), repeat=dim - 1):
            coords = [0] * dim
            for a, t in zip(tang, tcoords):
                coords[a] = t
            for side, q in ((0, 0), (1, n - 1)):
                g = sc.dirichlet.get((axis, side))
                if g is None:
                    continue
                coords[axis] = q
                c = host_index(n, dim, coords)
                diag[c] += t_half[c]
                rhs[c] += t_half[c] * g
            for q in range(1, n):
                if (axis, q, tuple(tcoords)) in face_to_cell:
                    continue  # fractured face: host cells meet the fracture through interfaces only
                coords[axis] = q - 1
                cl = host_index(n, dim, coords)
                coords[axis] = q
                cr = host_index(n, dim, coords)
                tl, tr = t_half[cl], t_half[cr]
                couple(cl, cr, tl * tr / (tl + tr))

    # ---- fracture facets that are not intersections ----------------------------------
    for (direction, pt), inc in plain:
        bnd = _on_boundary(n, dim, pt, skip=direction)
        if bnd is not None:
            g = sc.dirichlet.get(bnd)
            if g is not None:
                for f, tau, _ in inc:
                    diag[off_f + f] += tau
                    rhs[off_f + f] += tau * g
            continue
        if len(inc) == 2:
            (f, tf, _), (g2, tg, _) = inc
            if tf + tg > 0.0:
                couple(off_f + f, off_f + g2, tf * tg / (tf + tg))
        # one incident cell: no-flux tip

    # ---- line cells: neighbours along the line, and line ends on the boundary ------------
    if dim == 3:
        for v, inc in ends.items():
            bnd = _on_boundary(n, dim, v)
            if bnd is not None:
                g = sc.dirichlet.get(bnd)
                if g is not None:
                    for i, _ in inc:
                        diag[off_i + i] += tau_line[i]
                        rhs[off_i + i] += tau_line[i] * g
                continue
            if len({d for _, d in inc}) >= 2:
                continue  # a point: handled by its interfaces
            if len(inc) == 2:
                (i, _), (j, _) = inc
                ti, tj = tau_line[i], tau_line[j]
                if ti + tj > 0.0:
                    couple(off_i + i, off_i + j, ti * tj / (ti + tj))

    # ---- interfaces -------------------------------------------------------------------
    for e, (hi, lo, res) in enumerate(ifaces):
        r = n_cells + e
        rows.extend((hi, lo, r, r, r))
        cols.extend((r, r, hi, lo, r))
        vals.extend((1.0, -1.0, -1.0, 1.0, res))

    if sc.source is not None:
        rhs[:n_host] += np.asarray(sc.source, dtype=np.float64) * h ** dim

    rows.extend(range(n_cells))
    cols.extend(range(n_cells))
    vals.extend(diag[:n_cells].tolist())
    A = sp.coo_matrix((vals, (rows, cols)), shape=(n_tot, n_tot)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    part = np.zeros(n_tot, dtype=np.int32)
    part[n_cells:] = 1
    # cell centres (grid units of h) of every pressure unknown, for the pins
    cen = np.zeros((n_cells, dim))
    for c in range(n_host):
        r = c
        for a in range(dim):
            cen[c, a] = r % n + 0.5
            r //= n
    for f, (fi, t) in enumerate(cells):
        fr = sc.fractures[fi]
        tang = [a for a in range(dim) if a != fr.axis]
        cen[off_f + f, fr.axis] = fr.index
        for a, tt in zip(tang, t):
            cen[off_f + f, a] = tt + 0.5
    for i, (d, pt) in enumerate(inter_keys):
        cen[off_i + i] = pt
        if d >= 0:
            cen[off_i + i, d] += 0.5
    for p, v in enumerate(point_keys):
        cen[off_p + p] = v
    # dimension of each unknown's subdomain (an interface: its lower side's)
    labels = np.zeros(n_tot, dtype=np.int32)
    labels[:n_host] = dim
    labels[off_f:off_i] = dim - 1
    labels[off_i:off_p] = dim - 2
    labels[off_p:n_cells] = dim - 3
    labels[n_cells:] = [labels[lo] for _, lo, _ in ifaces]
    info = {"host": n_host, "fracture": nf, "intersection": ni, "point": npt, "interface": n_if,
            "cells": n_cells, "centres": cen * h, "interfaces": [(hi, lo) for hi, lo, _ in ifaces],
            "labels": labels}
    return A, rhs, part, info
