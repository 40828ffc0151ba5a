"""Shared comparison of the device factorization with the oracle's (test helper)."""
import numpy as np

from oracle.rs import compression_block

U = np.finfo(np.float64).eps


def compare_skeletons(h, F, residual_every=1):
    """Skeleton sets equal on every box whose subtree has no tie; returns
    (#boxes compared, #boxes skipped because of a tie below or at them).

    T agrees with the oracle's to within the conditioning of R11 (up to 1/eps), and the
    device's T satisfies the ID column-residual bound on the oracle's own block M.
    """
    ks, sk = h.box_skeletons()
    t = F.tree
    tied = set()
    for b in sorted(F.records, key=lambda b: -t.depth[b]):
        r = F.records[b]
        if r.idr.first_tie >= 0 or r.idr.near_threshold or any(c in tied for c in t.children[b]):
            tied.add(b)
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
