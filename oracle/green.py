"""Green's functions and Nystrom matrix entries (oracle; test infrastructure only).

The discretized operator is A = c I + K W restricted to the nodes: for i != j,
A_ij = K(x_i, x_j) w_j (weights on the columns, as in the point-sum discretization of
Section 2.1, Example 1, and the trapezoid rule of Section 6.2), and A_ii = c + d_i with a
per-kernel diagonal rule d_i.  c is the identity coefficient of a second-kind equation
(c = -1/2 for the interior Dirichlet double-layer equation, eq. (2k-integral-eqn));
c = 0 gives a first-kind equation.

Kernels
-------
lap2d_sl   G(x,y) = -(1/2pi) log|x-y|                      eq. (2d-laplace)
lap2d_dl   dG/dnu_y = (x-y).nu_y / (2 pi |x-y|^2)          eq. (double-layer), 2D
lap3d_sl   G(x,y) = 1 / (4 pi |x-y|)                        eq. (3d-laplace)
helm2d_cfie  dG_k/dnu_y - i eta G_k, G_k = (i/4) H0(k|x-y|) eq. (2d-helmholtz) with the
             combined layer mentioned at the end of Section 3.2 (complex128)
helm3d_sl  G_k(x,y) = exp(i k |x-y|) / (4 pi |x-y|)        eq. (3d-helmholtz) (complex128)

Diagonal rules (the paper's own quadrature corrections are not reproducible here):
lap2d_dl   d_i = -kappa_i w_i / (4 pi): the limit of the double-layer kernel along a
           smooth curve.  Pinned by the Gauss-lemma row sums and the unit-circle closed form.
lap2d_sl   d_i = -(w_i / 2pi) log(w_i / 2pi): the diagonal term that makes the equispaced
           rule exact for the constant mode of the log singularity (sum_{j!=i} of
           log|2 sin(pi (i-j)/N)| equals log N).  Pinned by unit-circle eigenvalues 1/(2m).
lap3d_sl   d_i = sqrt(w_i / pi) / 2: the single-layer integral over a flat disc of area
           w_i centred at the node.  Pinned by S[1] -> 1 on the unit sphere.
helm3d_sl  d_i = (exp(i k R) - 1) / (2 i k), R = sqrt(w_i / pi): the same flat-disc
           integral of exp(i k r) / (4 pi r) (its k -> 0 limit is the lap3d_sl rule).
           Pinned by the unit sphere's eigenvalues i k j_n(k) h_n(k) (n = 0, 1) and the
           k -> 0 limit.
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np

KINDS = ("lap2d_sl", "lap2d_dl", "lap3d_sl", "helm2d_cfie", "helm3d_sl")
EULER_GAMMA = 0.57721566490153286061


@dataclass
class Problem:
    """A Nystrom system: nodes, weights and kernel, in some fixed node order."""

    kind: str
    points: np.ndarray                      # (N, dim)
    weights: np.ndarray                     # (N,)
    normals: Optional[np.ndarray] = None    # (N, dim), double-layer kernels
    curvature: Optional[np.ndarray] = None  # (N,), 2D double-layer diagonal
    identity: float = 0.0                   # c in c I + K W
    wavenumber: float = 0.0                 # Helmholtz only
    eta: float = 0.0                        # Helmholtz combined-field coupling

    def __post_init__(self):
        if self.kind not in KINDS:
            raise ValueError(f"unknown kernel {self.kind}")
        self.points = np.asarray(self.points, dtype=np.float64)
        self.weights = np.asarray(self.weights, dtype=np.float64)

    @property
    def dim(self) -> int:
        return int(self.points.shape[1])

    @property
    def n(self) -> int:
        return int(self.points.shape[0])

    @property
    def is_complex(self) -> bool:
        return self.kind in ("helm2d_cfie", "helm3d_sl")

    @property
    def dtype(self):
        return np.complex128 if self.is_complex else np.float64

    @property
    def log_kernel(self) -> bool:
        """Kernels whose 2D single-layer part grows like log|x| (constant mode invisible
        on a unit proxy circle)."""
        return self.kind in ("lap2d_sl", "helm2d_cfie")

    def permuted(self, perm: np.ndarray) -> "Problem":
        """Same problem with nodes reordered: new node i is old node perm[i]."""
        return Problem(self.kind, self.points[perm], self.weights[perm],
                       None if self.normals is None else self.normals[perm],
                       None if self.curvature is None else self.curvature[perm],
                       self.identity, self.wavenumber, self.eta)


def kernel(prob: Problem, tgt: np.ndarray, src: np.ndarray,
           src_normals: Optional[np.ndarray] = None) -> np.ndarray:
    """K(x_t, y_s) for all target/source pairs, shape (len(tgt), len(src)).

    ``src_normals`` are the unit normals at the sources (double-layer kernels only).
    Coincident target/source pairs give inf/nan; callers overwrite the diagonal.
    """
    tgt = np.atleast_2d(tgt)
    src = np.atleast_2d(src)
    diff = tgt[:, None, :] - src[None, :, :]          # x - y
    r2 = np.sum(diff * diff, axis=-1)
    with np.errstate(divide="ignore", invalid="ignore"):
        if prob.kind == "lap2d_sl":
            return -np.log(np.sqrt(r2)) / (2.0 * np.pi)
        if prob.kind == "lap3d_sl":
            return 1.0 / (4.0 * np.pi * np.sqrt(r2))
        if prob.kind == "lap2d_dl":
            dot = np.sum(diff * src_normals[None, :, :], axis=-1)
            return dot / (2.0 * np.pi * r2)
        if prob.kind == "helm2d_cfie":
            from scipy.special import hankel1
            r = np.sqrt(r2)
            k = prob.wavenumber
            dot = np.sum(diff * src_normals[None, :, :], axis=-1)
            dl = 0.25j * k * hankel1(1, k * r) * dot / r
            sl = 0.25j * hankel1(0, k * r)
            return dl - 1j * prob.eta * sl
        if prob.kind == "helm3d_sl":
            r = np.sqrt(r2)
            return np.exp(1j * prob.wavenumber * r) / (4.0 * np.pi * r)
    raise ValueError(prob.kind)


def diagonal(prob: Problem, idx: np.ndarray) -> np.ndarray:
    """A_ii for the nodes idx: identity coefficient plus the kernel's diagonal rule."""
    w = prob.weights[idx]
    if prob.kind == "lap2d_sl":
        d = -(w / (2.0 * np.pi)) * np.log(w / (2.0 * np.pi))
    elif prob.kind == "lap2d_dl":
        d = -prob.curvature[idx] * w / (4.0 * np.pi)
    elif prob.kind == "lap3d_sl":
        d = 0.5 * np.sqrt(w / np.pi)
    elif prob.kind == "helm2d_cfie":
        k = prob.wavenumber
        dl = -prob.curvature[idx] * w / (4.0 * np.pi)
        sl = w * (0.25j - (np.log(k / 2.0) + EULER_GAMMA) / (2.0 * np.pi)) \
            - (w / (2.0 * np.pi)) * np.log(w / (2.0 * np.pi))
        d = dl - 1j * prob.eta * sl
    elif prob.kind == "helm3d_sl":
        k = prob.wavenumber
        R = np.sqrt(w / np.pi)
        d = (np.exp(1j * k * R) - 1.0) / (2j * k)
    else:
        raise ValueError(prob.kind)
    return prob.identity + d


def block(prob: Problem, rows: np.ndarray, cols: np.ndarray) -> np.ndarray:
    """A(rows, cols) with A_ij = c delta_ij + K(x_i, x_j) w_j, diagonal rule where i == j."""
    rows = np.asarray(rows, dtype=np.int64)
    cols = np.asarray(cols, dtype=np.int64)
    nrm = None if prob.normals is None else prob.normals[cols]
    a = kernel(prob, prob.points[rows], prob.points[cols], nrm) * prob.weights[cols][None, :]
    a = a.astype(prob.dtype, copy=False)
    ii, jj = np.nonzero(rows[:, None] == cols[None, :])
    if ii.size:
        a[ii, jj] = diagonal(prob, rows[ii])
    return a
