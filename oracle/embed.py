"""Forward compressed operator and its sparse embedding (oracle).

Section 2, eq. (compressed-representation) and eq. (sparse-embedding), and Section 3.4,
eq. (multilevel-embedding): after compression, A ~= A_eps with

    S_d ~= D_d + L_d S_{d-1} R_d         (one level, index set V_d -> V_{d-1})

where V_d are the DOFs active when depth d is compressed (S at the finest depth is
A itself), D_d is block diagonal over the depth-d boxes (the blocks S_d(J_B, J_B)),
L_d, R_d are the interpolation operators of those boxes, DOFs of leaves coarser than
d pass through unchanged (L = R = I, no diagonal part), and S_{d-1} is S_d restricted
to the surviving DOFs with the depth-d boxes' own skeleton-skeleton blocks removed.
The multilevel embedding stacks these one-level systems:

    [ D_d  L_d   0      ] [ x_d     ]   [ b ]
    [ R_d   0   -I      ] [ y_d     ] = [ 0 ]
    [  0   -I   S_{d-1} ] [ x_{d-1} ]   [ 0 ]

with S_0 the dense root block.  Solving this sparse system is the route the paper
takes (with a sparse LU); it is an independent check of the telescoping inverse.
"""
from __future__ import annotations

import numpy as np
import scipy.sparse as sp

from .green import block
from .rs import RSFactor


def _levels(F: RSFactor):
    """Per compressed depth (finest first): V_d, the boxes, and V_{d-1}."""
    t = F.tree
    leaves = [b for b in range(t.nbox) if t.is_leaf(b)]
    out = []
    for d in range(t.maxdepth, 0, -1):
        boxes = t.boxes_at(d)
        coarse = [np.arange(t.begin[b], t.end[b]) for b in leaves if t.depth[b] < d]
        coarse = np.concatenate(coarse) if coarse else np.zeros(0, dtype=np.int64)
        V = np.concatenate([F.records[b].J for b in boxes] + [coarse])
        Vn = np.concatenate([F.records[b].skel for b in boxes] + [coarse])
        out.append((d, boxes, V, Vn, coarse))
    return out


def _zero_own_blocks(F: RSFactor, boxes, rows_idx: np.ndarray, mat: np.ndarray):
    """Remove from mat (indexed by rows_idx x rows_idx) each box's skeleton block."""
    pos = {int(g): i for i, g in enumerate(rows_idx)}
    for b in boxes:
        s = np.array([pos[int(g)] for g in F.records[b].skel], dtype=np.int64)
        mat[np.ix_(s, s)] = 0.0


def embedding(F: RSFactor):
    """Sparse multilevel embedding (CSC) in tree order and the size of the x block."""
    prob = F.prob
    levels = _levels(F)
    blocks = []      # list of (row_offset, col_offset, sparse block)
    off = 0          # offset of the current x_d block
    size = None
    if not levels:
        A = block(prob, np.arange(prob.n), np.arange(prob.n))
        return sp.csc_matrix(A), prob.n, np.arange(prob.n)
    order = None
    for li, (d, boxes, V, Vn, coarse) in enumerate(levels):
        order = V if order is None else order     # x_d is ordered as y_{d+1} was
        nV, nK = V.size, Vn.size
        pos = {int(g): i for i, g in enumerate(order)}
        # D_d: depth-d boxes' diagonal blocks of S_d
        Dd = sp.lil_matrix((nV, nV), dtype=prob.dtype)
        Ld = sp.lil_matrix((nV, nK), dtype=prob.dtype)
        Rd = sp.lil_matrix((nK, nV), dtype=prob.dtype)
        kcol = 0
        for b in boxes:
            rec = F.records[b]
            loc = np.array([pos[int(g)] for g in rec.J], dtype=np.int64)
            Dd[np.ix_(loc, loc)] = _offdiag_D(F, rec)
            k = rec.k
            s_loc, r_loc = loc[rec.idr.skel], loc[rec.idr.redund]
            for a in range(k):
                Ld[s_loc[a], kcol + a] = 1.0
                Rd[kcol + a, s_loc[a]] = 1.0
            if k and r_loc.size:
                for a in range(k):
                    for c in range(r_loc.size):
                        Ld[r_loc[c], kcol + a] = rec.idr.T[a, c]
                        Rd[kcol + a, r_loc[c]] = rec.idr.T[a, c]
            kcol += k
        for g in coarse:           # pass-through DOFs
            Ld[pos[int(g)], kcol] = 1.0
            Rd[kcol, pos[int(g)]] = 1.0
            kcol += 1
        if size is None:
            size = nV
        # x_d at off, y_d at off + nV, x_{d-1} at off + nV + nK
        blocks.append((off, off, Dd.tocsc()))
        blocks.append((off, off + nV, Ld.tocsc()))
        blocks.append((off + nV, off, Rd.tocsc()))
        blocks.append((off + nV, off + nV + nK, -sp.identity(nK, dtype=prob.dtype, format="csc")))
        blocks.append((off + nV + nK, off + nV, -sp.identity(nK, dtype=prob.dtype, format="csc")))
        off = off + nV + nK
        last_Vn, last_boxes = Vn, boxes
        order = Vn
    # root block S_0: A on the surviving DOFs without the depth-1 boxes' own blocks
    S0 = block(prob, last_Vn, last_Vn)
    _zero_own_blocks(F, last_boxes, last_Vn, S0)
    blocks.append((off, off, sp.csc_matrix(S0)))
    total = off + last_Vn.size
    E = sp.lil_matrix((total, total), dtype=prob.dtype)
    Ecoo = [sp.coo_matrix(m) for (_, _, m) in blocks]
    rows = np.concatenate([c.row + r0 for (r0, _, _), c in zip(blocks, Ecoo)])
    cols = np.concatenate([c.col + c0 for (_, c0, _), c in zip(blocks, Ecoo)])
    vals = np.concatenate([c.data for c in Ecoo])
    E = sp.csc_matrix((vals, (rows, cols)), shape=(total, total))
    return E, size, levels[0][2]


def _offdiag_D(F: RSFactor, rec):
    """Above the finest depth: S_d(J_B, J_B) = A between siblings, zero inside a child."""
    D = block(F.prob, rec.J, rec.J)
    for (_, lo, hi) in rec.child_segments:
        D[lo:hi, lo:hi] = 0.0
    return D


def embedding_solve(F: RSFactor, b: np.ndarray) -> np.ndarray:
    """Solve the multilevel sparse embedding with SuperLU; b and x in caller order."""
    from scipy.sparse.linalg import splu
    E, nV, V = embedding(F)
    t = F.tree
    bt = b[t.perm]
    rhs = np.zeros((E.shape[0],) + b.shape[1:], dtype=np.result_type(b.dtype, F.prob.dtype))
    pos = np.empty(t.n, dtype=np.int64)
    pos[V] = np.arange(V.size)
    rhs[:nV] = bt[V]
    sol = splu(E.tocsc()).solve(rhs)
    xt = np.empty(bt.shape, dtype=rhs.dtype)      # complex for a complex operator
    xt[V] = sol[:nV]
    x = np.empty_like(xt)
    x[t.perm] = xt
    return x


def compressed_matvec(F: RSFactor, x: np.ndarray) -> np.ndarray:
    """A_eps x by the telescoping forward representation (upward R, root S, downward L).

    Section 3.3: an upward pass applying R level by level, the top skeleton matrix,
    then a downward pass applying L and adding the diagonal blocks D.
    """
    levels = _levels(F)
    t = F.tree
    xt = x[t.perm]
    cur = xt[levels[0][2]]
    order = levels[0][2]
    up = []
    for li, (d, boxes, V, Vn, coarse) in enumerate(levels):
        xv = cur                                   # values on ``order``
        pos = {int(g): i for i, g in enumerate(order)}
        out_D = np.zeros_like(xv)
        z = []
        for b in boxes:
            rec = F.records[b]
            loc = np.array([pos[int(g)] for g in rec.J], dtype=np.int64)
            Db = _offdiag_D(F, rec)
            out_D[loc] += Db @ xv[loc]
            xs = xv[loc[rec.idr.skel]] + rec.idr.T @ xv[loc[rec.idr.redund]]
            z.append(xs)
        z.append(xv[np.array([pos[int(g)] for g in coarse], dtype=np.int64)])
        up.append((V, Vn, boxes, coarse, pos, out_D))
        cur = np.concatenate(z)
        order = Vn
    Vn, boxes = levels[-1][3], levels[-1][1]   # cur is ordered as Vn
    S0 = block(F.prob, Vn, Vn)
    _zero_own_blocks(F, boxes, Vn, S0)
    y = S0 @ cur
    for (V, Vn, boxes, coarse, pos, out_D) in reversed(up):
        yv = out_D.copy()
        off = 0
        for b in boxes:
            rec = F.records[b]
            k = rec.k
            loc = np.array([pos[int(g)] for g in rec.J], dtype=np.int64)
            ys = y[off:off + k]
            yv[loc[rec.idr.skel]] += ys
            yv[loc[rec.idr.redund]] += rec.idr.T.T @ ys
            off += k
        for g in coarse:
            yv[pos[int(g)]] += y[off]
            off += 1
        y = yv
    V0 = levels[0][2]
    outt = np.empty_like(xt)
    outt[V0] = y
    out = np.empty_like(outt)
    out[t.perm] = outt
    return out
