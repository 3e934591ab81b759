"""Vectorised two-point-flux assembly of the host/fracture system (eq. (4)).

This is the library-side workload builder: it turns a raw scenario (grid,
permeabilities, fracture geometry, boundary values, sources) into the CSR
matrix, right-hand side and host/fracture partition that ``mdp_setup`` /
``mdp_solve`` take.  It is written array-at-a-time (all faces of one axis,
all facets of all fractures) so that 4M-cell grids assemble in seconds.

Discretisation of the model of Section 2.1 (eqs. (1)-(3)), as used
throughout this library:
  * host half transmissibility t = 2 K h^(dim-1) / h; unfractured faces
    couple host cells harmonically;
  * a fractured face couples each side X to the fracture cell with
    1 / (1/t_X + a / (2 kappa h^(dim-1))) and has no host-host term;
  * fracture cells meet at facets (vertices in 2D, edges in 3D) with half
    transmissibility tau = 2 K_par a |e| / h; an interior facet with several
    incident cells couples every pair by tau_f tau_g / sum(tau); a single
    incident cell is a no-flux tip; a facet on a Dirichlet boundary ties each
    incident cell to the boundary value through tau;
  * Dirichlet host faces add t (and t g to the right-hand side); sources add
    f h^dim.
Unknowns: host cells (x fastest), then fracture cells (fracture order, first
tangential axis fastest).
"""

from __future__ import annotations

from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse as sp


def _frac_cells(sc):
    """Per fracture: (axis, index, tangential axes, t-coordinate arrays,
    k_par, kappa, aperture, first id)."""
    out = []
    nxt = sc.n ** sc.dim
    for fr in sc.fractures:
        tang = [a for a in range(sc.dim) if a != fr.axis]
        lens = [h - l for l, h in zip(fr.lo, fr.hi)]
        m = int(np.prod(lens))
        k = np.arange(m)
        coords = []
        rem = k
        for ax, (l, ln) in enumerate(zip(fr.lo, lens)):
            coords.append(l + rem % ln)
            rem = rem // ln
        out.append((fr, tang, coords, nxt))
        nxt += m
    return out, nxt


def assemble(sc, sources: Optional[List[np.ndarray]] = None):
    """Return (A csr FP64, B, part).  B is the right-hand side for
    ``sc.source`` (shape (N,)), or, when ``sources`` is given, one column per
    source field (shape (N, len(sources)))."""
    n, dim = sc.n, sc.dim
    h = 1.0 / n
    area = h ** (dim - 1)
    nh = n ** dim
    fcells, ntot = _frac_cells(sc)
    kh = np.asarray(sc.k_host, dtype=np.float64)
    t = 2.0 * kh * area / h
    shape = (n,) * dim  # numpy axis order (z, y, x)
    idx = np.arange(nh).reshape(shape)

    # fracture lookup per axis: id of the fracture cell on face (q, tangential...)
    face_id = [np.full((n + 1,) + (n,) * (dim - 1), -1, dtype=np.int64) for _ in range(dim)]
    for fr, tang, coords, first in fcells:
        sel = [fr.index] + [c for c in coords]
        ids = first + np.arange(coords[0].size)
        tgt = face_id[fr.axis]
        if np.any(tgt[tuple(sel)] >= 0):
            raise ValueError("two fracture cells on one host face")
        tgt[tuple(sel)] = ids

    rows, cols, vals = [], [], []
    d_idx, d_val, r_idx, r_val = [], [], [], []

    def add_pairs(u, v, T):
        rows.append(u)
        cols.append(v)
        vals.append(-T)
        rows.append(v)
        cols.append(u)
        vals.append(-T)
        d_idx.extend((u, v))
        d_val.extend((T, T))

    def add_dirichlet(c, T, g):
        d_idx.append(c)
        d_val.append(T)
        r_idx.append(c)
        r_val.append(T * g)

    for axis in range(dim):
        npax = dim - 1 - axis
        tang = [a for a in range(dim) if a != axis]
        # move the face axis first, tangential axes after in increasing order
        perm = [npax] + [dim - 1 - a for a in tang]
        cells = np.transpose(idx, perm)          # [q][t1][t2]
        per_face = n ** (dim - 1)                # cells per layer (explicit: n = 1 has no interior faces)
        left = cells[:-1].reshape(n - 1, per_face)  # cells q-1 for q = 1..n-1
        right = cells[1:].reshape(n - 1, per_face)
        # face_id is indexed [q][t1][t2] with t1 the first tangential axis
        fid = face_id[axis][1:n].reshape(n - 1, per_face)
        L, R, F = left.ravel(), right.ravel(), fid.ravel()
        plain = F < 0
        tl, tr = t[L[plain]], t[R[plain]]
        add_pairs(L[plain], R[plain], tl * tr / (tl + tr))
        if np.any(~plain):
            Lf, Rf, Ff = L[~plain], R[~plain], F[~plain]
            nrm = np.empty(Ff.size)
            for fr, tg, coords, first in fcells:
                if fr.axis != axis:
                    continue
                msk = (Ff >= first) & (Ff < first + coords[0].size)
                nrm[msk] = fr.aperture / (2.0 * fr.kappa * area)
            add_pairs(Lf, Ff, 1.0 / (1.0 / t[Lf] + nrm))
            add_pairs(Ff, Rf, 1.0 / (1.0 / t[Rf] + nrm))
        for side in (0, 1):
            g = sc.dirichlet.get((axis, side))
            if g is None:
                continue
            bc = (cells[0] if side == 0 else cells[-1]).ravel()
            add_dirichlet(bc, t[bc], g)

    # fracture facets: key = (direction + 1, point coordinates) packed in int64
    base = n + 1
    keys, ids, taus, bnd_axis, bnd_side = [], [], [], [], []
    emeas = 1.0 if dim == 2 else h
    for fr, tang, coords, first in fcells:
        m = coords[0].size
        tau = 2.0 * fr.k_par * fr.aperture * emeas / h
        fid = first + np.arange(m)
        for mi, bm in enumerate(tang):
            others = [(mo, bo) for mo, bo in enumerate(tang) if bo != bm]
            direction = others[0][1] if others else -1
            for s in (0, 1):
                pt = [None] * dim
                pt[fr.axis] = np.full(m, fr.index)
                pt[bm] = coords[mi] + s
                for mo, bo in others:
                    pt[bo] = coords[mo]
                key = np.full(m, direction + 1, dtype=np.int64)
                for a in range(dim):
                    key = key * base + pt[a]
                keys.append(key)
                ids.append(fid)
                taus.append(np.full(m, tau))
                # boundary facet: its coordinate along bm hits 0 or n
                ba = np.where((pt[bm] == 0) | (pt[bm] == n), bm, -1)
                bnd_axis.append(ba)
                bnd_side.append((pt[bm] == n).astype(np.int64))
    if keys:
        key = np.concatenate(keys)
        fid = np.concatenate(ids)
        tau = np.concatenate(taus)
        bax = np.concatenate(bnd_axis)
        bsd = np.concatenate(bnd_side)
        on_b = bax >= 0
        for (a, sd), g in sc.dirichlet.items():
            msk = on_b & (bax == a) & (bsd == sd)
            add_dirichlet(fid[msk], tau[msk], g)
        key, fid, tau = key[~on_b], fid[~on_b], tau[~on_b]
        order = np.argsort(key, kind="stable")
        key, fid, tau = key[order], fid[order], tau[order]
        uk, start, cnt = np.unique(key, return_index=True, return_counts=True)
        tot = np.repeat(np.add.reduceat(tau, start) if tau.size else tau, cnt)
        maxc = int(cnt.max()) if cnt.size else 0
        for d in range(1, maxc):
            same = np.zeros(key.size, dtype=bool)
            same[:-d] = key[:-d] == key[d:]
            i = np.flatnonzero(same)
            j = i + d
            ok = tot[i] > 0
            i, j = i[ok], j[ok]
            add_pairs(fid[i], fid[j], tau[i] * tau[j] / tot[i])

    diag = np.bincount(np.concatenate(d_idx), weights=np.concatenate(d_val), minlength=ntot) \
        if d_idx else np.zeros(ntot)
    rhs_dir = np.bincount(np.concatenate(r_idx), weights=np.concatenate(r_val), minlength=ntot) \
        if r_idx else np.zeros(ntot)
    rows.append(np.arange(ntot))
    cols.append(np.arange(ntot))
    vals.append(diag)
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(ntot, ntot)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    part = np.zeros(ntot, dtype=np.int32)
    part[nh:] = 1

    vol = h ** dim
    if sources is None:
        b = rhs_dir.copy()
        if sc.source is not None:
            b[:nh] += np.asarray(sc.source, dtype=np.float64) * vol
        return A, b, part
    B = np.repeat(rhs_dir[:, None], len(sources), axis=1)
    for k, f in enumerate(sources):
        if f is not None:
            B[:nh, k] += np.asarray(f, dtype=np.float64) * vol
    return A, B, part
