"""Brute-force dense matrix and dense LU solve (oracle).

The plain definition the recursive-skeletonization solve approximates: A x = b with the
full N x N Nystrom matrix (Section 2), solved by Gaussian elimination with partial
pivoting.  Section 5 bounds the distance of the compressed solution to this one by
2 eps kappa / (1 - eps kappa).
"""
from __future__ import annotations

import numpy as np
from scipy.linalg import lu_factor, lu_solve

from .green import Problem, block


def matrix(prob: Problem) -> np.ndarray:
    idx = np.arange(prob.n)
    return block(prob, idx, idx)


def solve(prob: Problem, b: np.ndarray) -> np.ndarray:
    return lu_solve(lu_factor(matrix(prob)), b)


def matvec_rows(prob: Problem, rows: np.ndarray, x: np.ndarray, chunk: int = 2048) -> np.ndarray:
    """(A x)[rows] without forming A: used for residuals at sizes where A does not fit."""
    rows = np.asarray(rows, dtype=np.int64)
    out = np.zeros((rows.size,) + x.shape[1:], dtype=np.result_type(x.dtype, prob.dtype))
    cols = np.arange(prob.n)
    for lo in range(0, prob.n, chunk):
        c = cols[lo:lo + chunk]
        out += block(prob, rows, c) @ x[lo:lo + chunk]
    return out
