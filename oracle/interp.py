"""Interpolative decomposition by column-pivoted Householder QR (oracle).

Section 2.2: a rank-k ID writes A ~= B P where B holds k columns of A (the skeleton
columns) and P contains the k x k identity, with ||A - B P|| of the order of
sigma_{k+1}; the rank is chosen adaptively to a relative precision eps.  The paper
cites both a deterministic O(kmn) algorithm and a randomized one; this oracle uses the
deterministic route, column-pivoted QR in the Businger-Golub form:

* step j: pivot = the remaining column whose remaining part (rows j..m-1) has the
  largest 2-norm, recomputed from the current matrix (no norm downdating); exact ties
  go to the lowest original column index;
* stop at the first j with |R_jj| <= eps |R_00| (|R_jj| is that largest norm), so the
  rank k is the number of pivots with |R_jj| > eps |R_00|; a zero matrix has k = 0;
* with R11 the leading k x k triangle and R12 the next n-k columns,
  T = R11^{-1} R12 (k x (n-k)), so that A[:, rest] ~= A[:, skel] T.

The skeleton set s and the redundant set r are then each sorted ascending and T is
permuted to that order.

For comparisons with another implementation (the paper fixes no tie rule): two correct
Householder QRs of the same block differ by rounding, and the norms they recompute at a
step may differ by up to the backward error of Householder QR, of the order of m u
|R_00| in absolute terms (u the unit roundoff) -- small relative to the first pivots,
large relative to pivots near eps |R_00| when eps is small.  A pivot step is therefore
reported as tied when the two largest remaining norms differ by at most
1e-10 x the larger + 2 m u |R_00|, and the rank as near-threshold when |R_kk| or
|R_{k+1,k+1}| lies within 1e-10 eps |R_00| + 2 m u |R_00| of eps |R_00|.  Where
neither happens, the pivot order and the rank do not depend on rounding, and two
implementations must choose the same skeletons.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_triangular

TIE_RTOL = 1e-10
UNIT_ROUNDOFF = np.finfo(np.float64).eps / 2.0


def rounding_floor(m: int, r00: float) -> float:
    """Absolute width below which two norms of an m-row block are not told apart."""
    return 2.0 * m * UNIT_ROUNDOFF * r00


@dataclass
class IDResult:
    k: int
    skel: np.ndarray       # sorted local column indices (k,)
    redund: np.ndarray     # sorted local column indices (n-k,)
    T: np.ndarray          # (k, n-k), rows follow skel, columns follow redund
    pivots: np.ndarray     # original column indices in pivot order (n,)
    rdiag: np.ndarray      # |R_jj| for the pivot steps taken, plus the stopping value
    first_tie: int         # first tied pivot step (-1 if none among the k steps)
    near_threshold: bool


def cpqr_id(M: np.ndarray, eps: float, floor_rows: int = 0) -> IDResult:
    """floor_rows: row count for the rounding width of the tie rule (default M's own; a
    sketched block carries the rounding of the sum over the original block's rows)."""
    A = np.array(M, dtype=np.result_type(M.dtype, np.float64), copy=True)
    m, n = A.shape
    mf = max(m, floor_rows)
    perm = np.arange(n)
    rdiag = []
    first_tie = -1
    k = min(m, n)
    r00 = 0.0
    for j in range(min(m, n)):
        norms = np.sqrt(np.sum(np.abs(A[j:, j:]) ** 2, axis=0))
        best = norms.max()
        cand = np.nonzero(norms == best)[0]
        p = j + cand[np.argmin(perm[j + cand])]
        if j == 0:
            r00 = best
        rdiag.append(best)
        if best == 0.0 or best <= eps * r00:
            k = j
            break
        if first_tie < 0 and norms.size > 1:
            second = np.partition(norms, -2)[-2]
            if best - second <= TIE_RTOL * best + rounding_floor(mf, r00):
                first_tie = j
        # swap the pivot column into position j
        A[:, [j, p]] = A[:, [p, j]]
        perm[[j, p]] = perm[[p, j]]
        # Householder reflector H = I - 2 v v^* mapping A[j:, j] to a multiple of e_1
        x = A[j:, j].copy()
        alpha = np.linalg.norm(x)
        phase = x[0] / abs(x[0]) if x[0] != 0 else 1.0
        v = x.copy()
        v[0] += phase * alpha
        v /= np.linalg.norm(v)
        A[j:, j:] -= 2.0 * np.outer(v, v.conj() @ A[j:, j:])
    near = False
    if r00 > 0.0:
        thr = eps * r00
        for val in rdiag[max(0, k - 1):k + 1]:
            if abs(val - thr) <= TIE_RTOL * thr + rounding_floor(mf, r00):
                near = True
    R11 = np.triu(A[:k, :k])
    R12 = A[:k, k:]
    T = solve_triangular(R11, R12) if k > 0 else np.zeros((0, n - k), dtype=A.dtype)
    skel_p = perm[:k]
    red_p = perm[k:]
    so = np.argsort(skel_p, kind="stable")
    ro = np.argsort(red_p, kind="stable")
    return IDResult(k, skel_p[so], red_p[ro], T[so][:, ro], perm.copy(),
                    np.array(rdiag), first_tie, near)


# ---------------------------------------------------------------------------------
# Randomized ID (Section 2.2: the ID may be computed from a random sketch of the block,
# as in the paper's own code).  The block M (m x n) is compressed through its row sketch
# Y = Omega M with Omega an ell x m matrix of random signs, ell = min(m, n + oversample);
# the ID of Y (the column-pivoted QR above, with its rank rule) gives the skeletons and
# T.  When ell = m no sketch is taken (Y = M).  Omega's entries come from the SplitMix64
# counter-based generator (published by Steele, Lea and Flood, "Fast splittable
# pseudorandom number generators", OOPSLA 2014), so any implementation reproduces them
# exactly: entry (a, i) for box b is +1 or -1 by the top bit of
#     splitmix64(seed xor (b << 40) xor (a << 20) xor i).

_GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)


def splitmix64(x: np.ndarray) -> np.ndarray:
    """SplitMix64 output for the counters x (uint64 array): the generator's state after
    one increment by the golden gamma, mixed."""
    z = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = z + _GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def sketch_signs(box: int, rows: int, cols: int, seed: int) -> np.ndarray:
    """The rows x cols sign matrix Omega of box ``box`` (float64 entries +-1)."""
    a = np.arange(rows, dtype=np.uint64)[:, None]
    i = np.arange(cols, dtype=np.uint64)[None, :]
    ctr = (np.uint64(seed) ^ (np.uint64(box) << np.uint64(40)) ^ (a << np.uint64(20)) ^ i)
    top = splitmix64(ctr) >> np.uint64(63)
    return 1.0 - 2.0 * top.astype(np.float64)


def sketch_rows(m: int, n: int, oversample: int) -> int:
    return min(m, n + oversample)


def randomized_id(M: np.ndarray, eps: float, box: int, seed: int, oversample: int) -> IDResult:
    """ID of M through its row sketch (see above); the result refers to M's columns."""
    m, n = M.shape
    ell = sketch_rows(m, n, oversample)
    if ell >= m:
        return cpqr_id(M, eps)
    Y = sketch_signs(box, ell, m, seed) @ M
    return cpqr_id(Y, eps, floor_rows=m)
