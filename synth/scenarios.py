"""Raw scenario descriptions for fractured porous media on Cartesian grids.

Geometry conventions (shared vocabulary only, no arithmetic of the method):

* The domain is the unit square (dim 2) or unit cube (dim 3) with ``n`` cells
  per side.  Host cell ``(i, j[, k])`` has linear index ``i + n*j (+ n*n*k)``
  (x fastest).
* A fracture lies on host faces.  ``axis`` is the axis normal to it and
  ``index`` (1..n-1) the face plane along that axis: the faces between host
  cells ``index-1`` and ``index``.  ``lo``/``hi`` give the covered cell range
  (half open) along each tangential axis, tangential axes in increasing order.
* Fracture cells are numbered after all host cells: fracture by fracture in
  list order, inside a fracture over its tangential cell indices with the
  first tangential axis fastest.
* ``dirichlet`` maps ``(axis, side)`` (side 0 = low, 1 = high) to a boundary
  pressure; every other boundary is no-flux.
* ``source`` (optional) is a host source density per host cell.

The parameter ranges follow the paper's experiments: tangential and normal
fracture permeabilities from 1e-4 to 1e4 and unit matrix permeability
(Section 4, Table 1); the 3D case uses a unit cube with nine fracture planes
(Section 4.2).  The paper's benchmark geometries themselves are not used;
these generators are stand-ins with the same kind of structure.
"""

from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional, Tuple

import numpy as np


@dataclass
class Fracture:
    axis: int
    index: int
    lo: Tuple[int, ...]
    hi: Tuple[int, ...]
    k_par: float
    kappa: float
    aperture: float

    def n_cells(self) -> int:
        m = 1
        for a, b in zip(self.lo, self.hi):
            m *= b - a
        return m


@dataclass
class Scenario:
    dim: int
    n: int
    k_host: np.ndarray
    fractures: List[Fracture]
    dirichlet: Dict[Tuple[int, int], float]
    source: Optional[np.ndarray] = None
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n_host(self) -> int:
        return self.n ** self.dim

    @property
    def n_frac(self) -> int:
        return sum(f.n_cells() for f in self.fractures)

    @property
    def n_total(self) -> int:
        return self.n_host + self.n_frac

    def with_source(self, source: Optional[np.ndarray], name_suffix: str = "") -> "Scenario":
        return Scenario(self.dim, self.n, self.k_host, self.fractures, dict(self.dirichlet),
                        source, self.name + name_suffix, dict(self.meta))


def _x_dirichlet() -> Dict[Tuple[int, int], float]:
    return {(0, 0): 1.0, (0, 1): 0.0}


def grid_2d_four_lines(n: int = 32, k_par: float = 1e4, kappa: float = 1e4,
                       aperture: float = 1e-4) -> Scenario:
    """Unit square, unit host permeability, four full-length grid-aligned lines
    at x = 1/4, 3/4 and y = 1/4, 3/4, pressure 1 on x = 0 and 0 on x = 1."""
    if n % 4 != 0:
        raise ValueError("n must be a multiple of 4")
    fr = []
    for axis in (0, 1):
        for q in (n // 4, 3 * n // 4):
            fr.append(Fracture(axis, q, (0,), (n,), k_par, kappa, aperture))
    return Scenario(2, n, np.ones(n * n), fr, _x_dirichlet(),
                    name=f"2d-four-lines-n{n}-K{k_par:g}-k{kappa:g}")


def _lognormal(n_cells: int, seed: int, sigma: float) -> np.ndarray:
    z = np.random.default_rng(seed).standard_normal(n_cells)
    return np.exp(sigma * z)


def regular_3d(n: int = 100, k_par: float = 1e4, kappa: float = 1e4, seed: int = 0,
               sigma: float = 1.0, aperture: float = 1e-4,
               planes: Optional[List[Tuple[int, int]]] = None) -> Scenario:
    """Unit cube with (by default) nine full fracture planes, three per axis at
    face indices round(n/4), round(n/2), round(3n/4); log-normal host
    permeability exp(sigma*z), z standard normal drawn with ``seed`` in host
    cell order; pressure 1 on x = 0 and 0 on x = 1."""
    if planes is None:
        qs = [int(round(n * t)) for t in (0.25, 0.5, 0.75)]
        planes = [(axis, q) for axis in range(3) for q in qs]
    fr = [Fracture(axis, q, (0, 0), (n, n), k_par, kappa, aperture) for axis, q in planes]
    k = _lognormal(n ** 3, seed, sigma) if sigma > 0 else np.ones(n ** 3)
    return Scenario(3, n, k, fr, _x_dirichlet(),
                    name=f"3d-regular-n{n}-K{k_par:g}-k{kappa:g}-s{seed}",
                    meta={"seed": seed, "sigma": sigma})


def _loguniform(rng: np.random.Generator, lo_exp: float = -4.0, hi_exp: float = 4.0) -> float:
    return float(10.0 ** rng.uniform(lo_exp, hi_exp))


def random_2d(seed: int, n_range: Tuple[int, int] = (64, 512), max_segments: int = 20,
              aperture: float = 1e-4) -> Scenario:
    """Uneven 2D system: side n uniform in n_range, 1..max_segments random
    grid-aligned segments (normal axis by a fair coin, line index, start and
    length uniform), clipped to the domain; segments that would share a host
    face with an earlier segment are dropped.  Each segment gets its own
    log-uniform K_par and kappa in [1e-4, 1e4]."""
    rng = np.random.default_rng([seed, 2])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    n_seg = int(rng.integers(1, max_segments + 1))
    used = set()
    fr = []
    for _ in range(n_seg):
        axis = int(rng.integers(0, 2))
        line = int(rng.integers(1, n))
        start = int(rng.integers(0, n))
        length = int(rng.integers(-(-n // 8), n + 1))
        stop = min(start + length, n)
        k_par = _loguniform(rng)
        kappa = _loguniform(rng)
        faces = {(axis, line, t) for t in range(start, stop)}
        if stop <= start or faces & used:
            continue
        used |= faces
        fr.append(Fracture(axis, line, (start,), (stop,), k_par, kappa, aperture))
    return Scenario(2, n, np.ones(n * n), fr, _x_dirichlet(),
                    name=f"2d-random-s{seed}-n{n}-f{len(fr)}", meta={"seed": seed})


def random_3d(seed: int, n_range: Tuple[int, int] = (40, 160), aperture: float = 1e-4) -> Scenario:
    """Uneven 3D system: side n uniform in n_range, a random subset (3..9) of
    the nine full planes at round(n*{1/4,1/2,3/4}) per axis, each plane with
    its own log-uniform K_par and kappa in [1e-4, 1e4]; unit host permeability."""
    rng = np.random.default_rng([seed, 3])
    n = int(rng.integers(n_range[0], n_range[1] + 1))
    qs = [int(round(n * t)) for t in (0.25, 0.5, 0.75)]
    all_planes = [(axis, q) for axis in range(3) for q in qs]
    m = int(rng.integers(3, 10))
    pick = sorted(rng.choice(9, size=m, replace=False).tolist())
    fr = []
    for p in pick:
        axis, q = all_planes[p]
        fr.append(Fracture(axis, q, (0, 0), (n, n), _loguniform(rng), _loguniform(rng), aperture))
    return Scenario(3, n, np.ones(n ** 3), fr, _x_dirichlet(),
                    name=f"3d-random-s{seed}-n{n}-p{m}", meta={"seed": seed})


def tiny_2d(n: int = 8, seed: int = 0, k_par: float = 1.0, kappa: float = 1.0,
            aperture: float = 1e-2, sigma: float = 0.5) -> Scenario:
    """Small 2D case for dense checks: one full line x = 1/2, one partial line
    on y with an interior tip, crossing it (a T/X junction), log-normal host."""
    half = n // 2
    fr = [Fracture(0, half, (0,), (n,), k_par, kappa, aperture),
          Fracture(1, max(1, n // 4), (1,), (n - 1,), k_par * 2.0, kappa * 0.5, aperture)]
    k = _lognormal(n * n, seed, sigma)
    return Scenario(2, n, k, fr, _x_dirichlet(), name=f"2d-tiny-n{n}-s{seed}")


def tiny_3d(n: int = 6, seed: int = 0, k_par: float = 1.0, kappa: float = 1.0,
            aperture: float = 1e-2, sigma: float = 0.5) -> Scenario:
    """Small 3D case: three mutually intersecting planes (one per axis), one of
    them partial so that it has interior tips."""
    q = n // 2
    fr = [Fracture(0, q, (0, 0), (n, n), k_par, kappa, aperture),
          Fracture(1, q, (0, 0), (n, n), k_par * 3.0, kappa, aperture),
          Fracture(2, max(1, n // 3), (1, 1), (n - 1, n - 2), k_par, kappa * 2.0, aperture)]
    k = _lognormal(n ** 3, seed, sigma)
    return Scenario(3, n, k, fr, _x_dirichlet(), name=f"3d-tiny-n{n}-s{seed}")


def host_sources(sc: Scenario, seed: int, lo: float = -1.0, hi: float = 1.0) -> np.ndarray:
    """Host source density, uniform in [lo, hi) per host cell."""
    return np.random.default_rng([seed, 7]).uniform(lo, hi, sc.n_host)


def random_vector(size: int, seed: int) -> np.ndarray:
    """Standard-normal FP64 vector (e.g. a residual fed to one preconditioner
    application)."""
    return np.random.default_rng([seed, 11]).standard_normal(size)
