"""Recursive skeletonization: proxy compression, compressed inverse and solve (oracle).

Follows the paper step by step, in its notation:

Compression (Section 3.1, eq. (multilevel-compression)), level by level from the
finest boxes to the root.  All boxes of one depth are compressed against the same
matrix (the one-level scheme of Section 3.1 compresses every block row and column of
one matrix); boxes of a depth are therefore processed against a snapshot of the DOFs
still active when that depth starts.  For a box B at depth d:

* J_B = its nodes (leaf) or the concatenation of its children's skeletons (Section 3.1,
  "regroup"), each ascending, children in code order;
* proxy compression (Section 3.2): the far field is replaced by a proxy circle
  (sphere in 3D) of radius rho = 1.5 * side centred on the box, discretized by
  ``proxy_points`` points; near DOFs are the active DOFs outside J_B at distance
  < rho from the centre; the block compressed is
      M_B = [ A(N_B, J_B) ; A(J_B, N_B)^T ; K(Gamma, J_B) W_B ; (K(J_B, Gamma) W_Gamma)^T
              (; charge row ; constant row  for log kernels) ]
  so one ID gives both the outgoing and the incoming skeletons (one joint skeleton set
  per box, which keeps Lambda square);
* ID of M_B (module ``interp``) gives k, skeletons s, redundant r and T; then
  L_B = [I ; T^T] and R_B = [I  T] in (s, r) order: A(r, far) ~= T^T A(s, far) and
  A(far, r) ~= A(far, s) T.

Factorization (Section 3.4, eqs. (compressed-inverse), (multilevel-inverse)), literal:
  D_B = A(J_B, J_B) at a leaf; above the leaves the diagonal block of the level's
  S-matrix, i.e. Lambda of each child on the diagonal and A(s_a, s_b) between siblings;
  Lambda = (R D^{-1} L)^{-1};  cD = D^{-1} - D^{-1} L Lambda R D^{-1};
  cL = D^{-1} L Lambda;  cR = Lambda R D^{-1};  the root block S (Lambda of the
  depth-1 boxes plus A between their skeletons) is LU-factored.
  A box that keeps every DOF (k = n) is not compressed: L = R = I, Lambda = D, cD = 0.

Solve: x = cD^(1) b + cL^(1) [ cD^(2) (cR^(1) b) + cL^(2) ( ... S^{-1} ... ) ]:
an upward pass applying cR per box, the root solve, and a downward pass
x_B = cD_B b_B + cL_B z_B.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import Dict, List, Optional

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from .green import Problem, block, kernel
from .interp import IDResult, cpqr_id, randomized_id
from .tree import Tree, build_tree


@dataclass
class Options:
    eps: float
    proxy_points: int = 64
    proxy_ratio: float = 1.5
    id_mode: str = "cpqr"         # "cpqr": ID of M_B; "sketch": ID of its row sketch
    sketch_seed: int = 0
    oversample: int = 16


@dataclass
class BoxRecord:
    box: int
    depth: int
    leaf: bool
    J: np.ndarray           # active DOFs (tree positions), ascending
    near: np.ndarray        # near DOFs (tree positions), ascending
    m: int
    idr: IDResult
    child_segments: List[tuple] = field(default_factory=list)   # (child, lo, hi) in J
    D: Optional[np.ndarray] = None
    Lam: Optional[np.ndarray] = None
    cD: Optional[np.ndarray] = None
    cL: Optional[np.ndarray] = None
    cR: Optional[np.ndarray] = None

    @property
    def n(self) -> int:
        return int(self.J.size)

    @property
    def k(self) -> int:
        return self.idr.k

    @property
    def skel(self) -> np.ndarray:
        return self.J[self.idr.skel]

    @property
    def redund(self) -> np.ndarray:
        return self.J[self.idr.redund]


def proxy_surface(dim: int, center: np.ndarray, radius: float, npx: int):
    """Proxy points, their outward unit normals and their quadrature weight.

    2D: npx equispaced points on the circle, weight 2 pi rho / npx.
    3D: npx Fibonacci points on the sphere (z_p = 1 - (2p+1)/npx, azimuth
    p pi (3 - sqrt 5)), weight 4 pi rho^2 / npx.
    """
    p = np.arange(npx, dtype=np.float64)
    if dim == 2:
        th = 2.0 * np.pi * p / npx
        u = np.stack([np.cos(th), np.sin(th)], axis=1)
        wt = 2.0 * np.pi * radius / npx
    else:
        z = 1.0 - (2.0 * p + 1.0) / npx
        rr = np.sqrt(np.maximum(0.0, 1.0 - z * z))
        ph = p * (np.pi * (3.0 - np.sqrt(5.0)))
        u = np.stack([rr * np.cos(ph), rr * np.sin(ph), z], axis=1)
        wt = 4.0 * np.pi * radius * radius / npx
    return center[None, :] + radius * u, u, wt


def compression_block(prob: Problem, J: np.ndarray, near: np.ndarray, center: np.ndarray,
                      radius: float, npx: int) -> np.ndarray:
    """M_B of the proxy compression (Section 3.2) for the DOFs J of one box."""
    rows = []
    if near.size:
        rows.append(block(prob, near, J))          # near DOFs as targets
        rows.append(block(prob, J, near).T)        # near DOFs as sources
    Y, nu, wg = proxy_surface(prob.dim, center, radius, npx)
    xs = prob.points[J]
    ns = None if prob.normals is None else prob.normals[J]
    pt = kernel(prob, Y, xs, ns) * prob.weights[J][None, :]     # proxies as targets
    ps = (kernel(prob, xs, Y, nu) * wg).T                      # proxies as sources
    rows += [pt, ps]
    if prob.log_kernel:
        scale = max(np.abs(pt).max(), np.abs(ps).max())
        wj = prob.weights[J]
        rows.append((scale * wj / wj.max())[None, :])          # total charge of the box
        rows.append(np.full((1, J.size), scale))               # constant incoming field
    return np.vstack(rows).astype(prob.dtype, copy=False)


def near_dofs(points: np.ndarray, active: np.ndarray, own: np.ndarray, center: np.ndarray,
              radius: float) -> np.ndarray:
    """Active DOFs outside ``own`` strictly inside the proxy radius, ascending."""
    diff = points[active] - center[None, :]
    d2 = np.sum(diff * diff, axis=1)
    inside = d2 < radius * radius
    cand = active[inside]
    return np.sort(cand[~np.isin(cand, own)])


def literal_factor(D: np.ndarray, idr: IDResult):
    """(Lambda, cD, cL, cR) of Section 3.4 for one box; local (s, r) index sets."""
    n = D.shape[0]
    k = idr.k
    if k == n:
        return D.copy(), np.zeros_like(D), np.eye(n, dtype=D.dtype), np.eye(n, dtype=D.dtype)
    L = np.zeros((n, k), dtype=D.dtype)
    R = np.zeros((k, n), dtype=D.dtype)
    L[idr.skel, np.arange(k)] = 1.0
    L[np.ix_(idr.redund, np.arange(k))] = idr.T.T
    R[np.arange(k), idr.skel] = 1.0
    R[np.ix_(np.arange(k), idr.redund)] = idr.T
    lu = lu_factor(D, check_finite=True)
    if np.any(np.diag(lu[0]) == 0):
        raise np.linalg.LinAlgError("singular diagonal block")
    Dinv = lu_solve(lu, np.eye(n, dtype=D.dtype))
    WL = Dinv @ L
    WR = R @ Dinv
    Lam = np.linalg.inv(R @ WL) if k > 0 else np.zeros((0, 0), dtype=D.dtype)
    cD = Dinv - WL @ Lam @ WR
    return Lam, cD, WL @ Lam, Lam @ WR


class RSFactor:
    """Compressed inverse of one problem (tree order internally, caller order at the API)."""

    def __init__(self, prob: Problem, tree: Tree, opts: Options):
        self.caller_prob = prob
        self.tree = tree
        self.opts = opts
        self.prob = prob.permuted(tree.perm)
        self.records: Dict[int, BoxRecord] = {}
        self.root_J: np.ndarray = np.zeros(0, dtype=np.int64)
        self.root_S: Optional[np.ndarray] = None
        self.root_lu = None
        self.root_segments: List[tuple] = []

    # -- compression and factorization ------------------------------------------------
    def _assemble_diag(self, J: np.ndarray, segs: List[tuple]) -> np.ndarray:
        D = block(self.prob, J, J)
        for (c, lo, hi) in segs:
            D[lo:hi, lo:hi] = self.records[c].Lam
        return D

    def _gather_children(self, b: int):
        segs, parts, off = [], [], 0
        for c in self.tree.children[b]:
            s = self.records[c].skel
            segs.append((c, off, off + s.size))
            parts.append(s)
            off += s.size
        J = np.concatenate(parts) if parts else np.zeros(0, dtype=np.int64)
        return J, segs

    def run(self):
        t, prob, o = self.tree, self.prob, self.opts
        leaves = [b for b in range(t.nbox) if t.is_leaf(b)]
        for d in range(t.maxdepth, 0, -1):
            level = t.boxes_at(d)
            Js, segs = {}, {}
            for b in level:
                if t.is_leaf(b):
                    Js[b] = np.arange(t.begin[b], t.end[b], dtype=np.int64)
                    segs[b] = []
                else:
                    Js[b], segs[b] = self._gather_children(b)
            coarse = [np.arange(t.begin[b], t.end[b]) for b in leaves if t.depth[b] < d]
            active = np.sort(np.concatenate([Js[b] for b in level] + coarse))
            for b in level:
                J = Js[b]
                radius = o.proxy_ratio * t.side[b]
                near = near_dofs(prob.points, active, J, t.center[b], radius)
                if J.size == 0:
                    idr = cpqr_id(np.zeros((0, 0)), o.eps)
                    M_rows = 0
                else:
                    M = compression_block(prob, J, near, t.center[b], radius, o.proxy_points)
                    if o.id_mode == "sketch":
                        idr = randomized_id(M, o.eps, b, o.sketch_seed, o.oversample)
                    else:
                        idr = cpqr_id(M, o.eps)
                    M_rows = M.shape[0]
                rec = BoxRecord(b, d, t.is_leaf(b), J, near, M_rows, idr, segs[b])
                self.records[b] = rec
            for b in level:       # factor after every box of the level is compressed
                rec = self.records[b]
                rec.D = self._assemble_diag(rec.J, rec.child_segments)
                rec.Lam, rec.cD, rec.cL, rec.cR = literal_factor(rec.D, rec.idr)
        # root
        if t.is_leaf(0):
            self.root_J = np.arange(t.n, dtype=np.int64)
            self.root_segments = []
        else:
            self.root_J, self.root_segments = self._gather_children(0)
        self.root_S = self._assemble_diag(self.root_J, self.root_segments)
        if self.root_J.size:
            self.root_lu = lu_factor(self.root_S)
            if np.any(np.diag(self.root_lu[0]) == 0):
                raise np.linalg.LinAlgError("singular root block")
        return self

    # -- inverse application -----------------------------------------------------------
    def solve(self, b: np.ndarray) -> np.ndarray:
        """x = A_eps^{-1} b, b in caller order, shape (N,) or (N, nrhs)."""
        t = self.tree
        vec = b.ndim == 1
        B = (b[:, None] if vec else b)[t.perm].astype(np.result_type(b.dtype, self.prob.dtype))
        X = np.zeros_like(B)
        bin_, cout = {}, {}
        for d in range(t.maxdepth, 0, -1):          # upward pass: c_B = cR_B b_B
            for bx in t.boxes_at(d):
                rec = self.records[bx]
                if rec.leaf:
                    bb = B[t.begin[bx]:t.end[bx]]
                else:
                    bb = np.concatenate([cout[c] for c in t.children[bx]], axis=0)
                bin_[bx] = bb
                cout[bx] = rec.cR @ bb
        if t.is_leaf(0):
            c_root = B
        else:
            c_root = np.concatenate([cout[c] for c in t.children[0]], axis=0)
        out = {}
        if self.root_J.size:
            out[0] = lu_solve(self.root_lu, c_root)
        else:
            out[0] = c_root
        if t.is_leaf(0):
            X[:] = out[0]
        for d in range(1, t.maxdepth + 1):          # downward pass
            for bx in t.boxes_at(d):
                rec = self.records[bx]
                p = t.parent[bx]
                psegs = self.root_segments if p == 0 else self.records[p].child_segments
                lo, hi = next((lo, hi) for (c, lo, hi) in psegs if c == bx)
                z = out[p][lo:hi]
                xb = rec.cD @ bin_[bx] + rec.cL @ z
                if rec.leaf:
                    X[t.begin[bx]:t.end[bx]] = xb
                else:
                    out[bx] = xb
        Y = np.empty_like(X)
        Y[t.perm] = X
        return Y[:, 0] if vec else Y

    # -- reporting ------------------------------------------------------------------
    def level_stats(self):
        rows = []
        t = self.tree
        for d in range(t.maxdepth, 0, -1):
            recs = [self.records[b] for b in t.boxes_at(d)]
            rows.append(dict(depth=d, boxes=len(recs),
                             n=sum(r.n for r in recs), k=sum(r.k for r in recs),
                             max_n=max((r.n for r in recs), default=0),
                             max_m=max((r.m for r in recs), default=0)))
        return rows

    @property
    def root_size(self) -> int:
        return int(self.root_J.size)

    def storage_doubles(self) -> int:
        tot = 0
        for r in self.records.values():
            tot += r.cD.size + r.cL.size + r.cR.size
        if self.root_S is not None:
            tot += self.root_S.size
        return tot

    def ties(self) -> List[int]:
        return [b for b, r in self.records.items()
                if r.idr.first_tie >= 0 or r.idr.near_threshold]


def factor(prob: Problem, eps: float, leaf_size: int = 64, proxy_points: int = 64,
           proxy_ratio: float = 1.5, tree: Optional[Tree] = None, id_mode: str = "cpqr",
           sketch_seed: int = 0, oversample: int = 16) -> RSFactor:
    """Build the tree (unless given), compress and factor; returns the RSFactor.
    id_mode "sketch" compresses each block through its random row sketch
    (interp.randomized_id) instead of the block itself."""
    if tree is None:
        tree = build_tree(prob.points, leaf_size)
    if id_mode not in ("cpqr", "sketch"):
        raise ValueError(id_mode)
    return RSFactor(prob, tree, Options(eps, proxy_points, proxy_ratio, id_mode, sketch_seed,
                                        oversample)).run()
