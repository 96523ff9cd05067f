"""Seeded synthetic microstructures and material parameters.

This module is shared input synthesis only: it writes the uint8 phase arrays
and the per-phase Lame parameters that both the oracle and the HIP path
consume.  It holds none of the homogenization method's arithmetic (no Green
operator, no FFT, no tensor-train work).

Conventions
-----------
* Periodic unit cell of side 1 discretised into N x N x N voxels, N = 2**n.
* The phase of voxel (i, j, k) is decided at its centre ((i+1/2)/N, ...)
  with the periodic minimum-image distance and a strict "<" (a voxel centre
  on a sphere surface is outside).  The paper samples grid functions on
  binary fractions (Sec. 4.3, binary discretisation); sampling at voxel
  centres keeps cubic symmetry of a centred sphere and avoids ties.
* Arrays are C-ordered with x slowest: ``phase[ix, iy, iz]``.  Reshaped to
  ``(2,)*3n`` this is the core order of the quantized tensor train (x bits,
  then y bits, then z bits, most significant bit first).
* Phase 0 is the matrix, phase 1.. are inclusions.
* Random microstructures follow the rejection rule of the paper's App. F:
  the whole set of spheres is redrawn when any pair overlaps.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Problem", "lame_from_young", "reference_medium", "centres",
    "sphere", "laminate", "fibres", "spheres", "random_spheres",
    "config_c0", "config_c1_laminate", "config_c1_sphere", "config_c2",
    "config_c3", "config_c3_structure", "config_c4", "homogeneous",
    "synthetic_train", "geometry", "SUITE_2D", "SUITE_3D", "SUITE_YOUNG_NU", "suite_lame",
]


def lame_from_young(E: float, nu: float) -> tuple[float, float]:
    """Isotropic (lambda, mu) from Young's modulus and Poisson ratio."""
    lam = E * nu / ((1.0 + nu) * (1.0 - 2.0 * nu))
    mu = E / (2.0 * (1.0 + nu))
    return float(lam), float(mu)


def reference_medium(lame: np.ndarray) -> tuple[float, float]:
    """Reference medium: midpoint of the extreme phase Lame parameters.

    ``lame`` has shape (nphase, 2) with columns (lambda, mu).  For two phases
    this is the arithmetic mean of the phase moduli.
    """
    lame = np.asarray(lame, dtype=np.float64)
    lam0 = 0.5 * (lame[:, 0].min() + lame[:, 0].max())
    mu0 = 0.5 * (lame[:, 1].min() + lame[:, 1].max())
    return float(lam0), float(mu0)


def centres(N: int) -> np.ndarray:
    """Voxel-centre coordinates (i + 1/2)/N along one axis."""
    return (np.arange(N, dtype=np.float64) + 0.5) / N


def _periodic_delta(a: np.ndarray, c: float) -> np.ndarray:
    d = np.abs(a - c)
    return np.minimum(d, 1.0 - d)


def sphere(N: int, radius: float, centre=(0.5, 0.5, 0.5)) -> np.ndarray:
    """One sphere (phase 1) in a matrix (phase 0)."""
    x = centres(N)
    dx = _periodic_delta(x, centre[0])[:, None, None]
    dy = _periodic_delta(x, centre[1])[None, :, None]
    dz = _periodic_delta(x, centre[2])[None, None, :]
    inside = dx * dx + dy * dy + dz * dz < radius * radius
    return inside.astype(np.uint8)


def spheres(N: int, cs: np.ndarray, radii: np.ndarray) -> np.ndarray:
    """Union of spheres (phase 1) in a matrix (phase 0)."""
    x = centres(N)
    out = np.zeros((N, N, N), dtype=bool)
    for c, r in zip(np.asarray(cs), np.asarray(radii)):
        dx = _periodic_delta(x, c[0])[:, None, None]
        dy = _periodic_delta(x, c[1])[None, :, None]
        dz = _periodic_delta(x, c[2])[None, None, :]
        out |= dx * dx + dy * dy + dz * dz < r * r
    return out.astype(np.uint8)


def laminate(N: int, axis: int = 0, fraction: float = 0.5) -> np.ndarray:
    """Layers normal to ``axis``: voxels with index >= N*(1-fraction) are phase 1."""
    idx = np.arange(N)
    layer = (idx >= int(round(N * (1.0 - fraction)))).astype(np.uint8)
    shape = [1, 1, 1]
    shape[axis] = N
    return np.broadcast_to(layer.reshape(shape), (N, N, N)).copy()


def fibres(N: int, cs2d, radius: float) -> np.ndarray:
    """Cylindrical fibres along z through the (x, y) centres ``cs2d``."""
    x = centres(N)
    out = np.zeros((N, N), dtype=bool)
    for c in cs2d:
        dx = _periodic_delta(x, c[0])[:, None]
        dy = _periodic_delta(x, c[1])[None, :]
        out |= dx * dx + dy * dy < radius * radius
    return np.broadcast_to(out[:, :, None], (N, N, N)).astype(np.uint8)


def _periodic_dist(a: np.ndarray, b: np.ndarray) -> float:
    d = np.abs(a - b)
    d = np.minimum(d, 1.0 - d)
    return float(np.sqrt((d * d).sum()))


def random_spheres(rng: np.random.Generator, count: int, rmin: float,
                   rmax: float, scale_to_vf: float | None = None,
                   max_tries: int = 10000, per_sphere: bool = False):
    """Seeded non-overlapping spheres: centres first, then radii.

    The whole set is redrawn when any pair is closer than the sum of radii
    (App. F rejection rule).  With ``scale_to_vf`` all radii are scaled by one
    common factor so that the analytic volume fraction equals that value
    before the overlap test.  ``per_sphere``: only the centre of a sphere
    that overlaps an earlier one is redrawn (random sequential addition), for
    dense sets where a whole non-overlapping set is practically never drawn.
    """
    if per_sphere:
        rs = rng.uniform(rmin, rmax, size=count)
        if scale_to_vf is not None:
            vf = (4.0 / 3.0) * math.pi * float((rs ** 3).sum())
            rs = rs * (scale_to_vf / vf) ** (1.0 / 3.0)
        cs = np.zeros((count, 3))
        for i in range(count):
            for _ in range(max_tries):
                c = rng.uniform(0.0, 1.0, size=3)
                if all(_periodic_dist(c, cs[j]) > rs[i] + rs[j] for j in range(i)):
                    cs[i] = c
                    break
            else:
                raise RuntimeError("random_spheres: no room for a sphere")
        return cs, rs
    for _ in range(max_tries):
        cs = rng.uniform(0.0, 1.0, size=(count, 3))
        rs = rng.uniform(rmin, rmax, size=count)
        if scale_to_vf is not None:
            vf = (4.0 / 3.0) * math.pi * float((rs ** 3).sum())
            rs = rs * (scale_to_vf / vf) ** (1.0 / 3.0)
        ok = True
        for i in range(count):
            for j in range(i + 1, count):
                if _periodic_dist(cs[i], cs[j]) <= rs[i] + rs[j]:
                    ok = False
                    break
            if not ok:
                break
        if ok:
            return cs, rs
    raise RuntimeError("random_spheres: no non-overlapping set found")


@dataclass
class Problem:
    """One homogenization problem: voxels, phase moduli, solver settings."""
    name: str
    n: int
    phase: np.ndarray            # uint8 (N, N, N), C order, x slowest
    young_nu: list               # [(E, nu)] per phase
    cap: int
    delta: float                 # rounding accuracy delta_acc
    tol: float                   # fixed-point tolerance delta_tol
    meta: dict = field(default_factory=dict)

    @property
    def N(self) -> int:
        return 1 << self.n

    @property
    def lame(self) -> np.ndarray:
        return np.array([lame_from_young(E, nu) for E, nu in self.young_nu],
                        dtype=np.float64)

    @property
    def lame0(self) -> tuple[float, float]:
        return reference_medium(self.lame)

    def volume_fraction(self, p: int = 1) -> float:
        return float((self.phase == p).mean())


def homogeneous(n: int, E: float = 3.0, nu: float = 0.25) -> Problem:
    N = 1 << n
    return Problem("homogeneous", n, np.zeros((N, N, N), np.uint8),
                   [(E, nu), (E, nu)], cap=8, delta=1e-12, tol=1e-12)


def config_c0(exact: bool = False) -> Problem:
    """16^3 centred sphere R=0.25, E 1/10, nu 0.3; cap 32, delta 1e-10, tol 1e-8.

    ``exact`` selects the untruncated reading (no rank cap, delta 1e-14).
    """
    n = 4
    p = Problem("c0_sphere16", n, sphere(1 << n, 0.25), [(1.0, 0.3), (10.0, 0.3)],
                cap=32, delta=1e-10, tol=1e-8)
    if exact:
        p.name = "c0_sphere16_exact"
        p.cap = 1 << 30
        p.delta = 1e-14
    return p


def config_c1_laminate(n: int = 6) -> Problem:
    """64^3 laminate normal to x, vf 0.5; matrix (1, 0.3), layer (100, 0.2)."""
    return Problem("c1_laminate64", n, laminate(1 << n, 0, 0.5),
                   [(1.0, 0.3), (100.0, 0.2)], cap=64, delta=1e-8, tol=1e-6)


def config_c1_sphere(n: int = 6) -> Problem:
    """64^3 centred sphere of analytic vf 0.2; matrix (1, 0.3), sphere (100, 0.2)."""
    R = (3.0 * 0.2 / (4.0 * math.pi)) ** (1.0 / 3.0)
    return Problem("c1_sphere64", n, sphere(1 << n, R), [(1.0, 0.3), (100.0, 0.2)],
                   cap=64, delta=1e-8, tol=1e-6, meta={"radius": R})


def config_c2(n: int = 8) -> Problem:
    """256^3 four z-fibres R=0.15 on the square lattice (1/4, 3/4)^2.

    Fibre (20, 0.25), matrix (1, 0.35); cap 64, delta 1e-8, tol 1e-6.
    """
    cs = [(0.25, 0.25), (0.25, 0.75), (0.75, 0.25), (0.75, 0.75)]
    return Problem(f"c2_fibres{1 << n}", n, fibres(1 << n, cs, 0.15),
                   [(1.0, 0.35), (20.0, 0.25)], cap=64, delta=1e-8, tol=1e-6)


_C3_CAP = {5: 16, 6: 32, 7: 64}


def config_c3_structure(i: int, master_seed: int = 0, grid_n: int | None = None) -> Problem:
    """Structure ``i`` of the batched workload (seed [master, i]).

    Draw order: grid n in {5, 6, 7}; sphere count in 1..8; centres; radii in
    [0.05, 0.2]; then inclusion E in [2, 50].  nu = 0.3 for both phases,
    matrix E = 1.  Cap by grid: 32^3 -> 16, 64^3 -> 32, 128^3 -> 64.
    ``grid_n`` replaces the drawn grid (the draw still happens, so the
    geometry and moduli of structure i are unchanged); its cap is then the
    largest structural rank of that grid (no binding).
    """
    rng = np.random.default_rng([master_seed, i])
    n = int(rng.choice([5, 6, 7]))
    if grid_n is not None:
        n = grid_n
    count = int(rng.integers(1, 9))
    cs, rs = random_spheres(rng, count, 0.05, 0.2)
    E_incl = float(rng.uniform(2.0, 50.0))
    cap = _C3_CAP.get(n) if grid_n is None else _structural_cap(n)
    return Problem(f"c3_{i:03d}_n{n}", n, spheres(1 << n, cs, rs),
                   [(1.0, 0.3), (E_incl, 0.3)], cap=cap, delta=1e-7,
                   tol=1e-5, meta={"count": count, "E_incl": E_incl})


def _structural_cap(n: int) -> int:
    """Largest bond rank of a strain train on a 2^n grid (Voigt core of
    dimension 6, then 3n binary cores)."""
    L = 3 * n + 1
    best = 1
    for k in range(1, L):
        best = max(best, min(6 * 2 ** (k - 1), 2 ** (L - k)))
    return best


def config_c3(count: int = 256, master_seed: int = 0) -> list:
    return [config_c3_structure(i, master_seed) for i in range(count)]


def config_c4(n: int = 10, seed: int = 0) -> Problem:
    """1024^3, 64 random spheres, radii U[0.02, 0.08] rescaled to vf 0.15
    (placed one by one: at this density a whole non-overlapping set is
    practically never drawn)."""
    rng = np.random.default_rng(seed)
    cs, rs = random_spheres(rng, 64, 0.02, 0.08, scale_to_vf=0.15, per_sphere=True)
    return Problem(f"c4_spheres{1 << n}", n, spheres(1 << n, cs, rs),
                   [(1.0, 0.3), (10.0, 0.3)], cap=128, delta=1e-6, tol=1e-4,
                   meta={"centres": cs, "radii": rs})


def synthetic_train(n: int, rank: int = 64, seed: int = 1) -> list:
    """Seeded random complex strain train on the 2^n grid: Voigt core of
    dimension 6, then 3n binary cores, every bond min(rank, structural),
    entries standard normal in real and imaginary parts.  Cores have shape
    (1, r_{k-1}, d_k, r_k) (a batch of one train); the TTO-apply
    measurement and the full-size checks draw the same train."""
    rng = np.random.default_rng(seed)
    dims = [6] + [2] * (3 * n)
    L = len(dims)
    ranks = [1] + [min(rank, int(np.prod(dims[:k])), int(np.prod(dims[k:]))) for k in range(1, L)] + [1]
    return [(rng.standard_normal((1, ranks[k], d, ranks[k + 1]))
             + 1j * rng.standard_normal((1, ranks[k], d, ranks[k + 1]))) for k, d in enumerate(dims)]


# ---------------------------------------------------------------------------
# The paper's geometry suite (Sec. 5 and App. F): the 2D geometries and
# their two 3D generalisations (a non-varying z component; the same view
# from every direction).  Phase 1 (grey) E = 29/3, phase 0 (white) E = 4/3,
# both nu = 1/3.
# ---------------------------------------------------------------------------
SUITE_YOUNG_NU = [(4.0 / 3.0, 1.0 / 3.0), (29.0 / 3.0, 1.0 / 3.0)]


def _grid(N: int, dim: int):
    x = centres(N)
    return np.meshgrid(*([x] * dim), indexing="ij")


def _spots_centres(rng: np.random.Generator, count: int, radius: float, dim: int,
                   max_tries: int = 10000) -> np.ndarray:
    """Centres of `count` equal non-overlapping discs / balls (the whole
    set redrawn on any overlap, App. F)."""
    for _ in range(max_tries):
        cs = rng.uniform(0.0, 1.0, size=(count, dim))
        if all(_periodic_dist(cs[i], cs[j]) > 2 * radius
               for i in range(count) for j in range(i + 1, count)):
            return cs
    raise RuntimeError("spots: no non-overlapping set found")


def _voronoi(N: int, dim: int, seeds: int, fraction: float, rng: np.random.Generator) -> np.ndarray:
    """Periodic Voronoi cells of `seeds` uniform points; cells are taken as
    inclusions in a random order until their volume reaches `fraction`
    (App. F: a fraction of the cells, Phi_vol = 0.9)."""
    pts = rng.uniform(0.0, 1.0, size=(seeds, dim))
    g = _grid(N, dim)
    best = np.full(g[0].shape, np.inf)
    cell = np.zeros(g[0].shape, dtype=np.int64)
    for s, p in enumerate(pts):
        d2 = sum(_periodic_delta(g[a], p[a]) ** 2 for a in range(dim))
        closer = d2 < best
        best[closer] = d2[closer]
        cell[closer] = s
    out = np.zeros(g[0].shape, dtype=np.uint8)
    vol = np.bincount(cell.ravel(), minlength=seeds) / cell.size
    acc = 0.0
    for s in rng.permutation(seeds):
        if acc >= fraction:
            break
        out[cell == s] = 1
        acc += vol[s]
    return out


def geometry(name: str, N: int, dim: int = 2, seed: int = 0) -> np.ndarray:
    """uint8 phase array (N,)*dim of a suite geometry.

    2D: laminate, square (side 1/2), circle (radius 0.3), checkerboard
    (4 x 4 tiles), spots (10 discs of radius 0.08), voronoi (32 cells,
    Phi_vol 0.9).  3D: the z-extrusions pillar, circular_pillar, fibres,
    reduced_checkerboard, laminate3; the same-from-every-direction box,
    sphere, checkerboard3, voronoi3.
    """
    rng = np.random.default_rng(seed)
    if dim == 2:
        X, Y = _grid(N, 2)
        if name == "laminate":
            return (X >= 0.5).astype(np.uint8)
        if name == "square":
            return ((np.abs(X - 0.5) < 0.25) & (np.abs(Y - 0.5) < 0.25)).astype(np.uint8)
        if name == "circle":
            return ((X - 0.5) ** 2 + (Y - 0.5) ** 2 < 0.09).astype(np.uint8)
        if name == "checkerboard":
            return ((np.floor(4 * X) + np.floor(4 * Y)) % 2).astype(np.uint8)
        if name == "spots":
            cs = _spots_centres(rng, 10, 0.08, 2)
            out = np.zeros((N, N), dtype=bool)
            for c in cs:
                out |= _periodic_delta(X, c[0]) ** 2 + _periodic_delta(Y, c[1]) ** 2 < 0.08 ** 2
            return out.astype(np.uint8)
        if name == "voronoi":
            return _voronoi(N, 2, 32, 0.9, rng)
        raise ValueError(f"unknown 2D geometry {name!r}")
    extrude = {"laminate3": "laminate", "pillar": "square", "circular_pillar": "circle",
               "fibres": "spots", "reduced_checkerboard": "checkerboard"}
    if name in extrude:
        g2 = geometry(extrude[name], N, 2, seed)
        return np.broadcast_to(g2[:, :, None], (N, N, N)).copy()
    X, Y, Z = _grid(N, 3)
    if name == "box":
        return ((np.abs(X - 0.5) < 0.25) & (np.abs(Y - 0.5) < 0.25) & (np.abs(Z - 0.5) < 0.25)).astype(np.uint8)
    if name == "sphere":
        return sphere(N, 0.3)
    if name == "checkerboard3":
        return ((np.floor(4 * X) + np.floor(4 * Y) + np.floor(4 * Z)) % 2).astype(np.uint8)
    if name == "voronoi3":
        return _voronoi(N, 3, 32, 0.9, rng)
    raise ValueError(f"unknown 3D geometry {name!r}")


SUITE_2D = ["laminate", "square", "circle", "checkerboard", "spots", "voronoi"]
SUITE_3D = ["laminate3", "pillar", "circular_pillar", "box", "sphere", "fibres",
            "reduced_checkerboard", "checkerboard3", "voronoi3"]


def suite_lame() -> np.ndarray:
    return np.array([lame_from_young(E, nu) for E, nu in SUITE_YOUNG_NU], dtype=np.float64)
