"""Seeded synthetic workloads shared by the CPU oracle and the GPU path.

This module only draws inputs: surface point clouds, wavenumbers, self-term
spacings and excitation vectors. It holds none of the preconditioner's
arithmetic, so both sides can use it without sharing any method code.

Every generator takes an explicit seed and uses ``numpy.random.default_rng``.

Geometries follow the synthetic stand-ins for the paper's RWG meshes
(Sec. 5 uses plates, cubes and closed bodies discretised at about 10 points
per wavelength); the scalar point kernel replaces the RWG Galerkin entries of
Eq. 7.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

__all__ = [
    "Workload", "fibonacci_sphere", "ellipsoid_area", "sphere_ellipsoid",
    "cube_surface", "plate_box", "plane_wave", "port_vector", "make_config",
    "CONFIGS", "tiny_cluster_points",
]


def fibonacci_sphere(n: int, rng: np.random.Generator, jitter: float = 1e-3,
                     axes=(1.0, 1.0, 1.0), center=(0.0, 0.0, 0.0)) -> np.ndarray:
    """Fibonacci lattice on the unit sphere, scaled by ``axes``, plus uniform
    jitter in [-jitter, jitter]^3 (no re-projection)."""
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rad = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (math.pi * (3.0 - math.sqrt(5.0)))
    p = np.stack([rad * np.cos(phi), rad * np.sin(phi), z], axis=1)
    p *= np.asarray(axes, dtype=np.float64)[None, :]
    if jitter > 0:
        p += rng.uniform(-jitter, jitter, size=p.shape)
    p += np.asarray(center, dtype=np.float64)[None, :]
    return p


def ellipsoid_area(a: float, b: float, c: float) -> float:
    """Thomsen's approximation of an ellipsoid's surface area (p = 1.6075)."""
    q = 1.6075
    return 4.0 * math.pi * (((a * b) ** q + (a * c) ** q + (b * c) ** q) / 3.0) ** (1.0 / q)


def sphere_ellipsoid(n: int, rng: np.random.Generator, jitter: float = 1e-3):
    """Unit sphere at the origin plus an ellipsoid with axes (1, 0.6, 0.3)
    centred at (2.5, 0, 0); points split in proportion to area."""
    a_s = 4.0 * math.pi
    a_e = ellipsoid_area(1.0, 0.6, 0.3)
    n_s = int(round(n * a_s / (a_s + a_e)))
    n_e = n - n_s
    ps = fibonacci_sphere(n_s, rng, jitter)
    pe = fibonacci_sphere(n_e, rng, jitter, axes=(1.0, 0.6, 0.3), center=(2.5, 0.0, 0.0))
    return np.concatenate([ps, pe], axis=0), a_s + a_e


def cube_surface(n: int, rng: np.random.Generator, edge: float = 2.0):
    """Uniform points on the surface of an axis-aligned cube centred at the
    origin: face uniform among 6, (u, v) uniform on the face."""
    half = edge / 2.0
    face = rng.integers(0, 6, size=n)
    uv = rng.uniform(-half, half, size=(n, 2))
    p = np.empty((n, 3), dtype=np.float64)
    axis = face // 2
    sign = np.where(face % 2 == 0, -half, half)
    for ax in range(3):
        m = axis == ax
        others = [d for d in range(3) if d != ax]
        p[m, ax] = sign[m]
        p[m, others[0]] = uv[m, 0]
        p[m, others[1]] = uv[m, 1]
    return p, 6.0 * edge * edge


def plate_box(n: int, rng: np.random.Generator, dims=(2.0, 2.0, 0.05)):
    """Uniform points on the surface of a thin box (a plate with thickness)."""
    dx, dy, dz = dims
    areas = np.array([dy * dz, dy * dz, dx * dz, dx * dz, dx * dy, dx * dy])
    total = float(areas.sum())
    face = rng.choice(6, size=n, p=areas / total)
    u = rng.uniform(-0.5, 0.5, size=n)
    v = rng.uniform(-0.5, 0.5, size=n)
    p = np.empty((n, 3), dtype=np.float64)
    half = np.array([dx, dy, dz]) / 2.0
    for f in range(6):
        m = face == f
        ax = f // 2
        others = [d for d in range(3) if d != ax]
        p[m, ax] = -half[ax] if f % 2 == 0 else half[ax]
        p[m, others[0]] = u[m] * 2 * half[others[0]]
        p[m, others[1]] = v[m] * 2 * half[others[1]]
    return p, total


def tiny_cluster_points(rng: np.random.Generator, n_per: int = 8, centers=None):
    """Small point clusters (for hand-sized tests): ``n_per`` points jittered
    around each centre."""
    if centers is None:
        centers = [(0.0, 0.0, 0.0), (1.0, 0.0, 0.0), (2.0, 0.0, 0.0), (3.0, 0.0, 0.0)]
    pts = []
    for c in centers:
        pts.append(np.asarray(c)[None, :] + rng.uniform(-0.2, 0.2, size=(n_per, 3)))
    return np.concatenate(pts, axis=0)


def plane_wave(points: np.ndarray, k: float, rng: np.random.Generator) -> np.ndarray:
    """Plane-wave excitation b_m = exp(-j k d.p_m) with d uniform on the sphere."""
    d = rng.normal(size=3)
    d /= np.linalg.norm(d)
    return np.exp(-1j * k * (points @ d))


def port_vector(n: int, rng: np.random.Generator) -> np.ndarray:
    """Port excitation: a unit vector at a seeded index."""
    b = np.zeros(n, dtype=np.complex128)
    b[int(rng.integers(0, n))] = 1.0
    return b


@dataclass
class Workload:
    name: str
    points: np.ndarray          # N x 3 float64, user order
    k: float                    # wavenumber 2*pi/lambda
    self_h: float               # h = sqrt(area / N)
    leaf_max: int
    aca_tol: float = 1e-4
    fill_tol: float = 1e-2
    ordering: str = "rcm"
    restart: int = 30
    tol: float = 1e-6
    rhs: np.ndarray = field(default=None)   # N x nrhs complex128 (column-major use)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])


def make_config(name: str, n: int | None = None, nrhs: int = 1, seed: int | None = None) -> Workload:
    """Build one of the named workloads.

    * ``c1``: Fibonacci unit sphere, N=1200, lambda=0.5, leaf<=32, GMRES(30).
    * ``c2``: sphere + ellipsoid, N=20000, lambda=0.1, leaf<=64, GMRES(50).
    * ``c3``: cube surface (edge 2), N=100000, lambda=0.05, leaf<=64, GMRES(100)
      (GMRES(20) stagnates there; 50 takes 797 steps, 100 takes 341).
    * ``plate``: thin plate 2 x 2 x 0.05 with lambda = 10 h.
    ``n`` overrides the point count (the wavelength is kept) for scaled-down
    cases with the same structure.
    """
    name = name.lower()
    if name == "c1":
        n = n or 1200
        rng = np.random.default_rng(1 if seed is None else seed)
        pts = fibonacci_sphere(n, rng)
        area = 4.0 * math.pi
        lam, leaf, restart = 0.5, 32, 30
    elif name == "c2":
        n = n or 20000
        rng = np.random.default_rng(2 if seed is None else seed)
        pts, area = sphere_ellipsoid(n, rng)
        lam, leaf, restart = 0.1, 64, 50
    elif name == "c3":
        n = n or 100000
        rng = np.random.default_rng(3 if seed is None else seed)
        pts, area = cube_surface(n, rng)
        lam, leaf, restart = 0.05, 64, 100
    elif name == "plate":
        n = n or 5985
        rng = np.random.default_rng(6 if seed is None else seed)
        pts, area = plate_box(n, rng)
        lam, leaf, restart = None, 32, 30
    else:
        raise ValueError(f"unknown workload {name}")
    h = math.sqrt(area / n)
    if lam is None:
        lam = 10.0 * h
    k = 2.0 * math.pi / lam
    rhs = np.stack([plane_wave(pts, k, rng) for _ in range(nrhs)], axis=1)
    return Workload(name=name, points=pts, k=k, self_h=h, leaf_max=leaf,
                    restart=restart, rhs=np.asfortranarray(rhs))


CONFIGS = ("c1", "c2", "c3", "plate")


def batch_geometries(count: int = 64, n_max: int = 40000, seed: int = 4, nrhs: int = 4, ppl: float = 3.2) -> list:
    """Many geometries for batched runs: the body is uniform over sphere,
    ellipsoid (axes 1, 0.6, 0.3), cube (edge 2) and plate box (2 x 2 x 0.05);
    N uniform in [2000, n_max]; leaf_max uniform in [24, 96]; lambda = ppl h
    (ppl points per wavelength: 3.2 is the density of the 100,000-point cube
    at lambda = 0.05); nrhs plane waves. Geometry i uses the child seed
    1000 * seed + i."""
    out = []
    top = np.random.default_rng(seed)
    kinds = top.integers(0, 4, size=count)
    ns = top.integers(2000, n_max + 1, size=count)
    leaves = top.integers(24, 97, size=count)
    for i in range(count):
        rng = np.random.default_rng(1000 * seed + i)
        n = int(ns[i])
        kind = int(kinds[i])
        if kind == 0:
            pts, area, name = fibonacci_sphere(n, rng), 4.0 * math.pi, "sphere"
        elif kind == 1:
            pts, area, name = fibonacci_sphere(n, rng, axes=(1.0, 0.6, 0.3)), ellipsoid_area(1.0, 0.6, 0.3), "ellipsoid"
        elif kind == 2:
            (pts, area), name = cube_surface(n, rng), "cube"
        else:
            (pts, area), name = plate_box(n, rng), "plate"
        h = math.sqrt(area / n)
        k = 2.0 * math.pi / (ppl * h)
        rhs = np.stack([plane_wave(pts, k, rng) for _ in range(nrhs)], axis=1)
        out.append(Workload(name=name, points=pts, k=k, self_h=h, leaf_max=int(leaves[i]), restart=30,
                            rhs=np.asfortranarray(rhs)))
    return out
