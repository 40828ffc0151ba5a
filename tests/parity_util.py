"""Shared comparison of the device factorization with the oracle's (test helper)."""
import numpy as np

from oracle.rs import compression_block

U = np.finfo(np.float64).eps


def identical_skeletons(h, F):
    """True if every compressed box has the oracle's rank and skeleton set (then both
    sides compress to the same A_eps, whatever the tie flags say)."""
    ks, sk = h.box_skeletons()
    for b, r in F.records.items():
        if ks[b] != r.k or not np.array_equal(np.sort(sk[b]), r.skel):
            return False
    return True


def uncertain_boxes(depth, children, own_tie, active, near):
    """Boxes whose compression block may legitimately differ between two correct
    implementations: a box is uncertain if its own pivot sequence or rank decision is
    tied, if a child is uncertain (its active set then may differ), or if one of its
    active or near DOFs may or may not be active at its depth -- a DOF of an uncertain
    box at a finer depth, whose skeleton choice decides whether it survives.

    depth, children: per box; own_tie: box -> bool for the compressed boxes; active(b):
    the box's active DOFs (array); near(b, dofs): True if a DOF of the set `dofs` is in
    box b's near field."""
    bad = set()
    pending = set()          # DOFs whose activity at the current depth is uncertain
    by_depth = {}
    for b in own_tie:
        by_depth.setdefault(int(depth[b]), []).append(b)
    for d in sorted(by_depth, reverse=True):
        level_bad = []
        for b in by_depth[d]:
            u = bool(own_tie[b]) or any(c in bad for c in children[b])
            if not u and pending:
                u = bool(pending.intersection(active(b).tolist())) or near(b, pending)
            if u:
                level_bad.append(b)
        for b in level_bad:
            bad.add(b)
            pending.update(active(b).tolist())
    return bad


def compare_skeletons(h, F, residual_every=1):
    """Skeleton sets equal on every box that no tie can reach (uncertain_boxes); returns
    (#boxes compared, #boxes skipped as uncertain).

    T agrees with the oracle's to within the conditioning of R11 (up to 1/eps), and the
    device's T satisfies the ID column-residual bound on the oracle's own block M.
    """
    ks, sk = h.box_skeletons()
    t = F.tree
    own = {b: (r.idr.first_tie >= 0 or r.idr.near_threshold) for b, r in F.records.items()}
    tied = uncertain_boxes(t.depth, t.children, own, lambda b: F.records[b].J,
                           lambda b, dofs: bool(dofs.intersection(F.records[b].near.tolist())))
    compared = 0
    for b, r in F.records.items():
        if b in tied:
            continue
        assert ks[b] == r.k, f"rank differs at box {b}: {ks[b]} vs {r.k}"
        assert np.array_equal(np.sort(sk[b]), r.skel), f"skeletons differ at box {b}"
        J, T = h.box_export(b)
        assert np.array_equal(J, r.J)
        if r.k and r.n - r.k:
            scale = max(np.abs(r.idr.T).max(), 1.0)
            cond = r.idr.rdiag[0] / r.idr.rdiag[r.k - 1]
            assert np.abs(T - r.idr.T).max() <= 1e3 * U * cond * scale, f"T differs at box {b}"
            if b % residual_every == 0:
                tr = F.tree
                M = compression_block(F.prob, r.J, r.near, tr.center[b],
                                      F.opts.proxy_ratio * tr.side[b], F.opts.proxy_points)
                res = M[:, r.idr.redund] - M[:, r.idr.skel] @ T
                bound = 2.0 * r.idr.rdiag[r.k] + 1e-13 * r.idr.rdiag[0]
                assert np.linalg.norm(res, axis=0).max() <= bound, f"ID residual at box {b}"
        compared += 1
    return compared, len(tied)


def to_device(b, dtype=None):
    """Column-major device copy of a host (n,) or (n, nrhs) array."""
    import torch
    B = torch.tensor(np.asfortranarray(b), dtype=dtype, device="cuda")
    if B.dim() == 2:
        B = B.t().contiguous().t()
    return B
