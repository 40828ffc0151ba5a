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
permuted to that order.  For comparisons, a pivot step is reported as tied when the
two largest remaining norms agree to a relative 1e-10, and the rank is reported as
near-threshold when |R_kk| or |R_{k+1,k+1}| lies within a relative 1e-10 of eps |R_00|.
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy.linalg import solve_triangular

TIE_RTOL = 1e-10


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


def cpqr_id(M: np.ndarray, eps: float) -> IDResult:
    A = np.array(M, dtype=np.result_type(M.dtype, np.float64), copy=True)
    m, n = A.shape
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
            if best - second <= TIE_RTOL * best:
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
            if abs(val - thr) <= TIE_RTOL * thr:
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
