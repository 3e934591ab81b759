"""Vectorised assembly of the mixed-dimensional system with interface-flux
unknowns: the block reading of eq. (4) in which Omega holds the pressures of
every subdomain (host cells, fracture cells, and the intersection lines and
points as subdomains of their own, Section 2.1) and Gamma the fluxes over
the interfaces between subdomains of adjacent dimension.

Rows (two-point fluxes on the uniform grid):
  * subdomain cell: eq. (1) -- tangential fluxes to its neighbours in the
    same subdomain, plus Lambda for every interface where it is the higher-
    dimensional side (eq. (3): an outflow through its face), minus Lambda
    where it is the lower side, equal to its source;
  * interface: eq. (2) divided by its transmissibility,
    Lambda / T - p_high + p_low = 0, so A_GG is diagonal, positive, and
    A_GO = -A_OG^T (the library never assumes A_OG = A_GO^T).
Transmissibilities: host half t = 2 K A / h (harmonic across an unfractured
face); fracture cells tau = 2 K_par a |e| / h toward a facet of measure |e|
(1 in 2D, h in 3D), harmonic between coplanar neighbours; line cells
tau = 2 K_par a^2 / h toward each end, harmonic between collinear
neighbours; an intersection takes the mean K_par, kappa, aperture of its
incident cells.  Interface laws in series with the higher cell's half
transmissibility: host-fracture 1/T = 1/t + a/(2 kappa A),
fracture-intersection 1/T = 1/tau + 1/(2 kappa |e|), line-point
1/T = 1/tau + 1/(2 kappa a).  Intersections are the interior facets where
fracture cells of two or more planes meet; points (3D) the interior
vertices where line cells of two or more directions meet; a single cell at
a facet is a no-flux tip; facets and line ends on Dirichlet faces are tied
to the boundary value.

Unknown order: host cells (x fastest), fracture cells (fracture order, first
tangential axis fastest), intersection cells by (direction, lower corner
vertex with x fastest), points by vertex, then the interfaces: host-fracture
(per fracture cell, the host cell below then above), fracture-intersection
(per intersection, incident fracture cells ascending), line-point (per
point, incident line cells ascending).  part = 0 for pressures, 1 for
fluxes.
"""

from __future__ import annotations

from typing import List, Optional

import numpy as np
import scipy.sparse as sp

from .tpfa import _frac_cells


def _groups(key):
    """Start offsets and lengths of the runs of equal values in sorted key."""
    if key.size == 0:
        return np.zeros(0, dtype=np.int64), np.zeros(0, dtype=np.int64)
    brk = np.flatnonzero(key[1:] != key[:-1]) + 1
    start = np.concatenate(([0], brk))
    return start, np.diff(np.concatenate((start, [key.size])))


def assemble_flux(sc, sources: Optional[List[np.ndarray]] = None):
    """Return (A csr FP64, B, part, info).  B is the right-hand side for
    ``sc.source`` (shape (N,)), or one column per entry of ``sources``;
    info counts each kind of unknown."""
    n, dim = sc.n, sc.dim
    h = 1.0 / n
    area = h ** (dim - 1)
    nh = n ** dim
    fcells, n_hf = _frac_cells(sc)
    nf = n_hf - nh
    kh = np.asarray(sc.k_host, dtype=np.float64)
    t = 2.0 * kh * area / h
    shape = (n,) * dim
    idx = np.arange(nh).reshape(shape)
    V = (n + 1) ** dim
    vstride = np.array([(n + 1) ** a for a in range(dim)], dtype=np.int64)
    emeas = 1.0 if dim == 2 else h

    cr, cc, cv = [], [], []      # symmetric couplings among cells (off-diagonal)
    d_idx, d_val = [], []        # cell diagonal
    r_idx, r_val = [], []        # Dirichlet right-hand side
    hi_l, lo_l, res_l = [], [], []  # interfaces in order: high cell, low cell, 1/T

    def couple(u, v, T):
        cr.extend((u, v))
        cc.extend((v, u))
        cv.extend((-T, -T))
        d_idx.extend((u, v))
        d_val.extend((T, T))

    def tie(c, T, g):
        d_idx.append(c)
        d_val.append(T)
        r_idx.append(c)
        r_val.append(T * g)

    # ---- host faces: unfractured faces couple host cells; fractured ones give
    # the host-fracture interfaces
    face_id = [np.full((n + 1,) + (n,) * (dim - 1), -1, dtype=np.int64) for _ in range(dim)]
    for fr, tang, coords, first in fcells:
        sel = [fr.index] + list(coords)
        tgt = face_id[fr.axis]
        if np.any(tgt[tuple(sel)] >= 0):
            raise ValueError("two fracture cells on one host face")
        tgt[tuple(sel)] = first + np.arange(coords[0].size)
    hf_lo = np.full(nf, -1, dtype=np.int64)
    hf_hi = np.full(nf, -1, dtype=np.int64)
    for axis in range(dim):
        npax = dim - 1 - axis
        tang = [a for a in range(dim) if a != axis]
        cells = np.transpose(idx, [npax] + [dim - 1 - a for a in tang])
        per_face = n ** (dim - 1)
        L = cells[:-1].reshape(n - 1, per_face).ravel()
        R = cells[1:].reshape(n - 1, per_face).ravel()
        F = face_id[axis][1:n].reshape(n - 1, per_face).ravel()
        plain = F < 0
        tl, tr = t[L[plain]], t[R[plain]]
        couple(L[plain], R[plain], tl * tr / (tl + tr))
        hf_lo[F[~plain] - nh] = L[~plain]
        hf_hi[F[~plain] - nh] = R[~plain]
        for side in (0, 1):
            g = sc.dirichlet.get((axis, side))
            if g is not None:
                bc = (cells[0] if side == 0 else cells[-1]).ravel()
                tie(bc, t[bc], g)
    nrm = np.empty(nf)
    for fr, tang, coords, first in fcells:
        nrm[first - nh:first - nh + coords[0].size] = fr.aperture / (2.0 * fr.kappa * area)
    fids = nh + np.arange(nf)
    hi_l.append(np.stack((hf_lo, hf_hi), axis=1).ravel())
    lo_l.append(np.repeat(fids, 2))
    res_l.append(np.stack((1.0 / t[hf_lo] + nrm, 1.0 / t[hf_hi] + nrm), axis=1).ravel())

    # ---- fracture facets --------------------------------------------------------
    keys, fidl, taul, plane, kpl, kal, apl, bax, bsd = [], [], [], [], [], [], [], [], []
    for fr, tang, coords, first in fcells:
        m = coords[0].size
        tau = 2.0 * fr.k_par * fr.aperture * emeas / h
        fid = first + np.arange(m)
        for mi, bm in enumerate(tang):
            others = [(mo, bo) for mo, bo in enumerate(tang) if bo != bm]
            direction = others[0][1] if others else -1
            for s in (0, 1):
                pt = [None] * dim
                pt[fr.axis] = np.full(m, fr.index, dtype=np.int64)
                pt[bm] = coords[mi] + s
                for mo, bo in others:
                    pt[bo] = coords[mo]
                vtx = sum(pt[a] * vstride[a] for a in range(dim))
                keys.append((direction + 1) * V + vtx)
                fidl.append(fid)
                taul.append(np.full(m, tau))
                plane.append(np.full(m, fr.axis * (n + 1) + fr.index))
                kpl.append(np.full(m, fr.k_par))
                kal.append(np.full(m, fr.kappa))
                apl.append(np.full(m, fr.aperture))
                bax.append(np.where((pt[bm] == 0) | (pt[bm] == n), bm, -1))
                bsd.append((pt[bm] == n).astype(np.int64))
    ni = npt = 0
    line_tau = line_dir = line_vtx = line_ka = line_ap = None
    if keys:
        key, fid, tau = np.concatenate(keys), np.concatenate(fidl), np.concatenate(taul)
        pl, kp, ka, ap = np.concatenate(plane), np.concatenate(kpl), np.concatenate(kal), np.concatenate(apl)
        ba, bs = np.concatenate(bax), np.concatenate(bsd)
        on_b = ba >= 0
        for (a, sd), g in sc.dirichlet.items():
            msk = on_b & (ba == a) & (bs == sd)
            tie(fid[msk], tau[msk], g)
        keep = ~on_b
        key, fid, tau, pl, kp, ka, ap = (x[keep] for x in (key, fid, tau, pl, kp, ka, ap))
        order = np.lexsort((fid, key))
        key, fid, tau, pl, kp, ka, ap = (x[order] for x in (key, fid, tau, pl, kp, ka, ap))
        start, cnt = _groups(key)
        tot = np.add.reduceat(tau, start) if key.size else tau
        # facets where cells of two or more planes meet (with some conduction) are intersections
        pmin = np.minimum.reduceat(pl, start) if key.size else pl
        pmax = np.maximum.reduceat(pl, start) if key.size else pl
        npl = np.where(pmin != pmax, 2, 1)
        inter = (npl >= 2) & (tot > 0.0)
        # plain facets with two coplanar cells: harmonic coupling
        two = (~inter) & (cnt == 2)
        s2 = start[two]
        tf, tg = tau[s2], tau[s2 + 1]
        ok = tf + tg > 0.0
        couple(fid[s2][ok], fid[s2 + 1][ok], tf[ok] * tg[ok] / (tf[ok] + tg[ok]))
        # intersection cells, in key order (direction, then vertex)
        ist, icn = start[inter], cnt[inter]
        ni = ist.size
        ikey = key[ist]
        grp = np.repeat(np.arange(ni), icn)
        mem = np.concatenate([np.arange(s, s + c) for s, c in zip(ist, icn)]) if ni else np.zeros(0, np.int64)
        off_i = nh + nf
        hi_l.append(fid[mem])
        lo_l.append(off_i + grp)
        res_l.append(1.0 / tau[mem] + 1.0 / (2.0 * ka[mem] * emeas))
        cnt_f = np.maximum(icn, 1).astype(np.float64)
        mean = lambda x: np.add.reduceat(x[mem], np.concatenate(([0], np.cumsum(icn)[:-1]))) / cnt_f \
            if ni else np.zeros(0)
        line_kp, line_ka, line_ap = mean(kp), mean(ka), mean(ap)
        line_dir = ikey // V - 1
        line_vtx = ikey % V
        line_tau = 2.0 * line_kp * line_ap * line_ap / h if dim == 3 else np.zeros(ni)

    # ---- 3D line cells: neighbours along the line, points, Dirichlet ends ---------
    if dim == 3 and ni:
        off_i = nh + nf
        li = np.concatenate((np.arange(ni), np.arange(ni)))
        vend = np.concatenate((line_vtx, line_vtx + vstride[line_dir]))
        ldir = np.concatenate((line_dir, line_dir))
        coord = (vend // vstride[ldir]) % (n + 1)  # the end's coordinate along the line
        bnd = (coord == 0) | (coord == n)
        for side, cval in ((0, 0), (1, n)):
            for a in range(dim):
                g = sc.dirichlet.get((a, side))
                if g is None:
                    continue
                msk = bnd & (ldir == a) & (coord == cval)
                tie(off_i + li[msk], line_tau[li[msk]], g)
        li, vend, ldir = li[~bnd], vend[~bnd], ldir[~bnd]
        order = np.lexsort((li, vend))
        li, vend, ldir = li[order], vend[order], ldir[order]
        start, cnt = _groups(vend)
        dmin = np.minimum.reduceat(ldir, start) if vend.size else ldir
        dmax = np.maximum.reduceat(ldir, start) if vend.size else ldir
        ispt = dmin != dmax
        two = (~ispt) & (cnt == 2)
        s2 = start[two]
        ta, tb = line_tau[li[s2]], line_tau[li[s2 + 1]]
        ok = ta + tb > 0.0
        couple(off_i + li[s2][ok], off_i + li[s2 + 1][ok], ta[ok] * tb[ok] / (ta[ok] + tb[ok]))
        pst, pcn = start[ispt], cnt[ispt]
        npt = pst.size
        if npt:
            pgrp = np.repeat(np.arange(npt), pcn)
            pmem = np.concatenate([np.arange(s, s + c) for s, c in zip(pst, pcn)])
            L = li[pmem]
            if np.any(line_tau[L] == 0.0):
                raise ValueError("a point joins a line cell without tangential conduction")
            hi_l.append(off_i + L)
            lo_l.append(off_i + ni + pgrp)
            res_l.append(1.0 / line_tau[L] + 1.0 / (2.0 * line_ka[L] * line_ap[L]))

    # ---- matrix ------------------------------------------------------------------------
    n_cells = nh + nf + ni + npt
    hi = np.concatenate(hi_l) if hi_l else np.zeros(0, np.int64)
    lo = np.concatenate(lo_l) if lo_l else np.zeros(0, np.int64)
    res = np.concatenate(res_l) if res_l else np.zeros(0)
    n_if = hi.size
    ntot = n_cells + n_if
    e = n_cells + np.arange(n_if)
    diag = np.bincount(np.concatenate(d_idx), weights=np.concatenate(d_val), minlength=n_cells) \
        if d_idx else np.zeros(n_cells)
    rows = np.concatenate([np.concatenate(cr) if cr else np.zeros(0, np.int64), np.arange(n_cells), hi, lo, e, e, e])
    cols = np.concatenate([np.concatenate(cc) if cc else np.zeros(0, np.int64), np.arange(n_cells), e, e, hi, lo, e])
    vals = np.concatenate([np.concatenate(cv) if cv else np.zeros(0), diag, np.ones(n_if), -np.ones(n_if),
                           -np.ones(n_if), np.ones(n_if), res])
    A = sp.coo_matrix((vals, (rows, cols)), shape=(ntot, ntot)).tocsr()
    A.sum_duplicates()
    A.sort_indices()
    part = np.zeros(ntot, dtype=np.int32)
    part[n_cells:] = 1
    rhs_dir = np.bincount(np.concatenate(r_idx), weights=np.concatenate(r_val), minlength=ntot) \
        if r_idx else np.zeros(ntot)
    # dimension of each unknown's subdomain (an interface: its lower side's),
    # for dimension-aware aggregation
    labels = np.empty(ntot, dtype=np.int32)
    labels[:nh] = dim
    labels[nh:nh + nf] = dim - 1
    labels[nh + nf:nh + nf + ni] = dim - 2
    labels[nh + nf + ni:n_cells] = dim - 3
    labels[n_cells:] = labels[lo]
    info = {"host": nh, "fracture": nf, "intersection": ni, "point": npt, "interface": n_if, "cells": n_cells,
            "labels": labels}
    vol = h ** dim
    if sources is None:
        b = rhs_dir.copy()
        if sc.source is not None:
            b[:nh] += np.asarray(sc.source, dtype=np.float64) * vol
        return A, b, part, info
    B = np.repeat(rhs_dir[:, None], len(sources), axis=1)
    for k, f in enumerate(sources):
        if f is not None:
            B[:nh, k] += np.asarray(f, dtype=np.float64) * vol
    return A, B, part, info
