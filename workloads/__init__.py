"""Seeded synthetic inputs: boundary geometries, quadrature weights and right-hand sides.

This module is shared by the CPU oracle, the tests and the benchmark. It holds
geometry and random-number generation only, none of the solver's arithmetic:
no Green's functions, no tree, no compression, no factorization.

Geometries (the paper's own test geometries are an ellipse and the unit sphere,
Section 6.2; the configurations used here replace them with a star-shaped curve,
random smooth curves and a quasi-uniform sphere of the same kind):

* ``star_curve``    r(t) = 1 + a cos(m t), equispaced parameter, trapezoid weights
* ``random_curve``  r(t) = 1 + sum_k a_k cos(k t + phi_k)
* ``ellipse``       semi-axes (a, b), equispaced parameter
* ``scatterer_curve``  r(t) = (2 + cos 3t) / 6 (the multiple-scattering example's body)
* ``fibonacci_sphere``  N quasi-uniform points on the unit sphere, equal-area weights

All arrays are float64.  Points are point-major, shape (N, dim).
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Optional

import numpy as np


@dataclass
class Geometry:
    """Discretized boundary: nodes, quadrature weights, outward normals, curvature."""

    points: np.ndarray                 # (N, dim)
    weights: np.ndarray                # (N,)
    normals: Optional[np.ndarray] = None   # (N, dim) outward unit normals
    curvature: Optional[np.ndarray] = None  # (N,) signed curvature (2D curves)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def dim(self) -> int:
        return int(self.points.shape[1])


def _polar_curve(n: int, r, dr, ddr, name: str, meta: dict) -> Geometry:
    """Closed curve x(t) = r(t) (cos t, sin t) sampled at t_j = 2 pi j / n.

    ``r``, ``dr``, ``ddr`` are callables giving r, r', r'' at an array of t.
    Weights are the trapezoid rule in t times the speed |x'(t)|; the normal
    (y', -x') / |x'| points outward for this counter-clockwise parameterization;
    the curvature is (r^2 + 2 r'^2 - r r'') / (r^2 + r'^2)^(3/2).
    """
    if n < 1:
        raise ValueError("n must be positive")
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    rv, d1, d2 = r(t), dr(t), ddr(t)
    c, s = np.cos(t), np.sin(t)
    x, y = rv * c, rv * s
    xp = d1 * c - rv * s
    yp = d1 * s + rv * c
    speed = np.sqrt(rv * rv + d1 * d1)
    w = speed * (2.0 * np.pi / n)
    nrm = np.stack([yp / speed, -xp / speed], axis=1)
    kap = (rv * rv + 2.0 * d1 * d1 - rv * d2) / (rv * rv + d1 * d1) ** 1.5
    pts = np.ascontiguousarray(np.stack([x, y], axis=1))
    return Geometry(pts, w, np.ascontiguousarray(nrm), kap, name, meta)


def star_curve(n: int, amp: float = 0.3, lobes: int = 5) -> Geometry:
    """Star r(t) = 1 + amp cos(lobes t)."""
    return _polar_curve(
        n,
        lambda t: 1.0 + amp * np.cos(lobes * t),
        lambda t: -amp * lobes * np.sin(lobes * t),
        lambda t: -amp * lobes * lobes * np.cos(lobes * t),
        "star", {"amp": amp, "lobes": lobes})


def scatterer_curve(n: int, center=(0.0, 0.0)) -> Geometry:
    """The scatterer of the paper's multiple-scattering example (Section 6.4):
    r(t) = (2 + cos 3t) / 6, shifted to ``center``."""
    g = _polar_curve(
        n,
        lambda t: (2.0 + np.cos(3.0 * t)) / 6.0,
        lambda t: -0.5 * np.sin(3.0 * t),
        lambda t: -1.5 * np.cos(3.0 * t),
        "scatterer", {"center": tuple(center)})
    g.points = g.points + np.asarray(center, dtype=np.float64)[None, :]
    return g


def random_curve(n: int, amps, phases) -> Geometry:
    """Smooth random curve r(t) = 1 + sum_{k>=1} amps[k-1] cos(k t + phases[k-1])."""
    amps = np.asarray(amps, dtype=np.float64)
    phases = np.asarray(phases, dtype=np.float64)
    ks = np.arange(1, len(amps) + 1, dtype=np.float64)

    def r(t):
        return 1.0 + (amps[None, :] * np.cos(np.outer(t, ks) + phases[None, :])).sum(1)

    def dr(t):
        return -(amps[None, :] * ks * np.sin(np.outer(t, ks) + phases[None, :])).sum(1)

    def ddr(t):
        return -(amps[None, :] * ks * ks * np.cos(np.outer(t, ks) + phases[None, :])).sum(1)

    return _polar_curve(n, r, dr, ddr, "random_curve", {"amps": amps, "phases": phases})


def circle(n: int, radius: float = 1.0) -> Geometry:
    return _polar_curve(n, lambda t: radius + 0.0 * t, lambda t: 0.0 * t,
                        lambda t: 0.0 * t, "circle", {"radius": radius})


def ellipse(n: int, a: float = 2.0, b: float = 1.0) -> Geometry:
    """Ellipse (a cos t, b sin t), equispaced t, trapezoid weights."""
    t = 2.0 * np.pi * np.arange(n, dtype=np.float64) / n
    x, y = a * np.cos(t), b * np.sin(t)
    xp, yp = -a * np.sin(t), b * np.cos(t)
    xpp, ypp = -a * np.cos(t), -b * np.sin(t)
    speed = np.sqrt(xp * xp + yp * yp)
    w = speed * (2.0 * np.pi / n)
    nrm = np.stack([yp / speed, -xp / speed], axis=1)
    kap = (xp * ypp - yp * xpp) / speed ** 3
    return Geometry(np.ascontiguousarray(np.stack([x, y], 1)), w,
                    np.ascontiguousarray(nrm), kap, "ellipse", {"a": a, "b": b})


def fibonacci_sphere(n: int, rotation: Optional[np.ndarray] = None) -> Geometry:
    """Quasi-uniform points on the unit sphere: z_i = 1 - (2i+1)/n, azimuth i*pi*(3-sqrt 5).

    Equal-area weights 4 pi / n; the normal is the point itself.
    """
    i = np.arange(n, dtype=np.float64)
    z = 1.0 - (2.0 * i + 1.0) / n
    rho = np.sqrt(np.maximum(0.0, 1.0 - z * z))
    phi = i * (np.pi * (3.0 - np.sqrt(5.0)))
    pts = np.stack([rho * np.cos(phi), rho * np.sin(phi), z], axis=1)
    if rotation is not None:
        pts = pts @ np.asarray(rotation, dtype=np.float64).T
    w = np.full(n, 4.0 * np.pi / n)
    return Geometry(np.ascontiguousarray(pts), w, np.ascontiguousarray(pts.copy()), None,
                    "fibonacci_sphere", {})


def random_rotation(rng: np.random.Generator) -> np.ndarray:
    """Haar-random 3x3 rotation (QR of a Gaussian matrix, sign-fixed)."""
    q, r = np.linalg.qr(rng.standard_normal((3, 3)))
    q = q * np.sign(np.diag(r))[None, :]
    if np.linalg.det(q) < 0:
        q[:, 0] = -q[:, 0]
    return q


def gaussian_rhs(n: int, nrhs: int, seed: int, complex_valued: bool = False) -> np.ndarray:
    """i.i.d. N(0,1) right-hand sides, column-major (Fortran order) (n, nrhs)."""
    rng = np.random.default_rng(seed)
    b = rng.standard_normal((n, nrhs))
    if complex_valued:
        b = b + 1j * rng.standard_normal((n, nrhs))
    return np.asfortranarray(b)


def random_curve_problem(p: int):
    """Member p of the family of random smooth curves used for many-problem batches.

    Draws, in order from default_rng(1000 + p): N ~ U{1024..16384}, a_k ~ U(0, 0.04)
    and phi_k ~ U[0, 2 pi) for k = 1..8, then one N(0,1) right-hand side.
    Returns (geometry, rhs).
    """
    rng = np.random.default_rng(1000 + p)
    n = int(rng.integers(1024, 16385))
    amps = rng.uniform(0.0, 0.04, 8)
    phases = rng.uniform(0.0, 2.0 * np.pi, 8)
    b = np.asfortranarray(rng.standard_normal((n, 1)))
    return random_curve(n, amps, phases), b


def diameter(points: np.ndarray) -> float:
    """Largest distance between two nodes (the diameter of the discretized boundary).

    The farthest pair of a point set lies on its convex hull, so only hull vertices are
    compared pairwise."""
    from scipy.spatial import ConvexHull
    pts = np.asarray(points, dtype=np.float64)
    if pts.shape[0] < pts.shape[1] + 2:
        cand = pts
    else:
        cand = pts[ConvexHull(pts).vertices]
    best = 0.0
    for lo in range(0, cand.shape[0], 1024):
        d = cand[lo:lo + 1024, None, :] - cand[None, :, :]
        best = max(best, float(np.sqrt((d * d).sum(axis=2)).max()))
    return best


def helmholtz_wavenumber(g: Geometry, wavelengths: float) -> float:
    """Wavenumber k with the given number of wavelengths across the domain: the width is
    the domain's diameter (the largest node-to-node distance; 2.4919 for the star
    curve), so k = 2 pi wavelengths / diameter (Section 6.1 counts wavelengths as
    k diam / (2 pi))."""
    return 2.0 * np.pi * wavelengths / diameter(g.points)


# Named workloads (sizes of the benchmark and parity configurations).
WORKLOADS = {
    "lap2d_dl_star_4096": dict(geom=("star", 4096), kind="lap2d_dl", eps=1e-9, leaf=64,
                               proxy=64, nrhs=1, seed=0),
    "lap2d_sl_star_65536": dict(geom=("star", 65536), kind="lap2d_sl", eps=1e-9, leaf=64,
                                proxy=64, nrhs=512, seed=1),
    "lap3d_sl_sphere_20480": dict(geom=("sphere", 20480), kind="lap3d_sl", eps=1e-6,
                                  leaf=128, proxy=512, nrhs=64, seed=2),
    # exterior combined field 1/2 I + D_k - i k S_k, 10 wavelengths across the star
    "helm2d_cfie_star_32768": dict(geom=("star", 32768), kind="helm2d_cfie", eps=1e-9,
                                   leaf=64, proxy=64, nrhs=1, seed=3, wavelengths=10.0,
                                   identity=0.5),
}


def proxy_count(kind: str, eps: float) -> int:
    """Proxy points per box: 64 on the circle down to eps = 1e-9, 96 beyond; 512 on the sphere."""
    if kind.startswith("lap3d"):
        return 512
    return 64 if eps >= 1e-9 else 96
