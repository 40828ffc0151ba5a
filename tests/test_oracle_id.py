"""Pins of the oracle's interpolative decomposition (CPU).

Checked against what the mathematics fixes: the exact column-residual bound of
column-pivoted QR, exact recovery of low-rank matrices, LAPACK's pivoted QR
(geqp3, via scipy) on untied inputs, and the singular-value bracket of an ID.
"""
import numpy as np
import pytest
from scipy.linalg import qr, svdvals

from oracle.interp import cpqr_id


def _lowrank(m, n, q, rng, decay=None):
    U, _ = np.linalg.qr(rng.standard_normal((m, q)))
    V, _ = np.linalg.qr(rng.standard_normal((n, q)))
    s = np.ones(q) if decay is None else decay ** np.arange(q)
    return (U * s) @ V.T


@pytest.mark.parametrize("seed", range(4))
def test_residual_columns_bounded_by_next_pivot(seed):
    # After k steps, M[:, r] - M[:, s] T = Q [0; R22], whose column norms are bounded
    # by the largest remaining column norm |R_{k+1,k+1}| <= eps |R_00|.
    rng = np.random.default_rng(seed)
    M = _lowrank(80, 50, 50, rng, decay=0.6)
    eps = 1e-7
    idr = cpqr_id(M, eps)
    assert 0 < idr.k < 50
    res = M[:, idr.redund] - M[:, idr.skel] @ idr.T
    bound = idr.rdiag[idr.k]
    assert np.all(np.linalg.norm(res, axis=0) <= bound * (1 + 1e-10) + 1e-14)
    assert bound <= eps * idr.rdiag[0]
    assert idr.rdiag[idr.k - 1] > eps * idr.rdiag[0]


def test_rdiag_nonincreasing_and_skeleton_columns_exact():
    rng = np.random.default_rng(7)
    M = rng.standard_normal((60, 40)) @ np.diag(0.8 ** np.arange(40))
    idr = cpqr_id(M, 1e-9)
    assert np.all(np.diff(idr.rdiag) <= 1e-12 * idr.rdiag[0])
    # the projection matrix P holds the identity on the skeleton columns
    P = np.zeros((idr.k, 40))
    P[:, idr.skel] = np.eye(idr.k)
    P[:, idr.redund] = idr.T
    approx = M[:, idr.skel] @ P
    assert np.array_equal(approx[:, idr.skel], M[:, idr.skel])


@pytest.mark.parametrize("q", [1, 5, 17])
def test_exact_low_rank_recovered(q):
    rng = np.random.default_rng(q)
    M = _lowrank(70, 45, q, rng)
    idr = cpqr_id(M, 1e-12)
    assert idr.k == q
    res = M[:, idr.redund] - M[:, idr.skel] @ idr.T
    assert np.abs(res).max() < 1e-13


@pytest.mark.parametrize("seed", range(5))
def test_pivots_match_lapack_geqp3(seed):
    rng = np.random.default_rng(100 + seed)
    M = rng.standard_normal((50, 30)) * (0.7 ** np.arange(30))[None, :]
    idr = cpqr_id(M, 0.0)
    _, R, piv = qr(M, pivoting=True, mode="economic")
    assert idr.k == 30
    assert list(idr.pivots) == list(piv)
    assert np.allclose(idr.rdiag[:30], np.abs(np.diag(R)), rtol=1e-12)


def test_id_error_bracketed_by_singular_values():
    # ||M - M_s P|| >= sigma_{k+1} always, and is within a modest factor of it.
    rng = np.random.default_rng(3)
    M = _lowrank(100, 60, 60, rng, decay=0.5)
    idr = cpqr_id(M, 1e-6)
    P = np.zeros((idr.k, 60))
    P[:, idr.skel] = np.eye(idr.k)
    P[:, idr.redund] = idr.T
    err = np.linalg.norm(M - M[:, idr.skel] @ P, 2)
    sv = svdvals(M)
    assert err >= sv[idr.k] * (1 - 1e-8)
    assert err <= 50 * sv[idr.k]


def test_degenerate_inputs():
    z = cpqr_id(np.zeros((10, 4)), 1e-9)
    assert z.k == 0 and z.T.shape == (0, 4) and list(z.redund) == [0, 1, 2, 3]
    e = cpqr_id(np.eye(4), 0.0)
    assert e.k == 4 and e.T.shape == (4, 0)
    # wide matrix: rank limited by the row count
    w = cpqr_id(np.random.default_rng(0).standard_normal((3, 8)), 0.0)
    assert w.k == 3


def test_exact_ties_break_to_lowest_original_index():
    M = np.zeros((4, 3))
    M[0, 2] = 2.0
    M[1, 0] = 2.0
    M[2, 1] = 1.0
    idr = cpqr_id(M, 0.0)
    assert list(idr.pivots[:2]) == [0, 2]
    assert idr.first_tie == 0


def test_complex_id():
    rng = np.random.default_rng(11)
    X = rng.standard_normal((40, 10)) + 1j * rng.standard_normal((40, 10))
    Y = rng.standard_normal((10, 30)) + 1j * rng.standard_normal((10, 30))
    A = X @ Y
    idr = cpqr_id(A, 1e-12)
    assert idr.k == 10
    res = A[:, idr.redund] - A[:, idr.skel] @ idr.T
    assert np.abs(res).max() < 1e-13 * np.abs(A).max()


def _orthogonal_columns(m, norms, seed):
    """m x n matrix whose columns are orthogonal with the given 2-norms: column-pivoted QR
    takes them in order of decreasing norm and |R_jj| equals the j-th largest norm (up to
    rounding)."""
    Q, _ = np.linalg.qr(np.random.default_rng(seed).standard_normal((m, len(norms))))
    return Q * np.asarray(norms)[None, :]


@pytest.mark.parametrize("rel,expect_k,expect_near", [
    (1e-12, 4, True),      # |R_33| just above eps |R_00|: kept, but within the band
    (-1e-12, 3, True),     # just below: dropped, and the stopping value is within it
    (1e-9, 4, True),       # 1e-15 from the threshold: inside the rounding floor
    (1e-7, 4, False),      # outside the band on either side
    (-1e-7, 3, False),
])
def test_near_threshold_flag(rel, expect_k, expect_near):
    # The rank rule keeps pivots with |R_jj| > eps |R_00|; a decision taken within
    # 1e-10 eps |R_00| + 2 m u |R_00| of the threshold (here 40 rows, |R_00| = 1: about
    # 8.9e-15) is flagged, since rounding may take it either way.
    eps = 1e-6
    norms = [1.0, 0.5, 0.25, eps * (1.0 + rel), 1e-9, 1e-10]
    M = _orthogonal_columns(40, norms, 5)
    idr = cpqr_id(M, eps)
    assert idr.k == expect_k
    assert idr.near_threshold is expect_near
    assert list(idr.pivots[:4]) == [0, 1, 2, 3]
    assert abs(idr.rdiag[3] - norms[3]) <= 1e-15


def test_near_threshold_clear_when_rank_gap_is_wide():
    # |R_kk| two orders of magnitude on either side of eps |R_00|: no flag.
    eps = 1e-3
    norms = [1.0, 0.9, 1e-1, 1e-5, 1e-7]
    M = _orthogonal_columns(30, norms, 9)
    idr = cpqr_id(M, eps)
    assert idr.k == 3
    assert idr.near_threshold is False


def test_tie_flag_uses_the_rounding_floor():
    # Orthogonal columns: at step 2 the two remaining norms are 1e-8 and 1e-8 (1 + 1e-7),
    # 1e-15 apart -- far more than a relative 1e-10 of either, but below the absolute
    # width 2 m u |R_00| (about 8.9e-15 for 40 rows) within which two Householder QRs
    # of this block may disagree.  The step is reported as tied.
    norms = [1.0, 0.5, 1e-8 * (1.0 + 1e-7), 1e-8, 1e-12]
    M = _orthogonal_columns(40, norms, 3)
    idr = cpqr_id(M, 1e-14)
    assert idr.first_tie == 2
    assert list(idr.pivots[:2]) == [0, 1]
    # well separated norms: no tie anywhere
    M2 = _orthogonal_columns(40, [1.0, 0.5, 1e-3, 0.5e-3, 1e-6], 4)
    assert cpqr_id(M2, 1e-9).first_tie == -1


def test_splitmix64_reference_outputs():
    # The generator's first three outputs from state 0 (the published reference values):
    # counters 0, gamma, 2 gamma.
    from oracle.interp import splitmix64
    g = 0x9E3779B97F4A7C15
    out = splitmix64(np.array([0, g, (2 * g) % (1 << 64)], dtype=np.uint64))
    assert [int(v) for v in out] == [0xE220A8397B1DCDAF, 0x6E789E6AA1B965F4, 0x06C45D188009454F]


def test_sketch_signs_balanced_and_reproducible():
    from oracle.interp import sketch_signs
    S = sketch_signs(7, 300, 2000, 12345)
    assert set(np.unique(S)) == {-1.0, 1.0}
    assert abs(S.mean()) < 0.01                    # 6e5 fair signs: sd 1.3e-3
    assert np.array_equal(S, sketch_signs(7, 300, 2000, 12345))
    assert not np.array_equal(S, sketch_signs(8, 300, 2000, 12345))
    # rows are nearly orthogonal (E[S S^T] = m I)
    G = S @ S.T / 2000.0
    assert np.abs(G - np.eye(300)).max() < 0.15


def test_randomized_id_exact_low_rank_and_identity_when_short():
    from oracle.interp import randomized_id
    rng = np.random.default_rng(3)
    A = rng.standard_normal((400, 12)) @ rng.standard_normal((12, 50))
    idr = randomized_id(A, 1e-12, box=5, seed=99, oversample=16)
    assert idr.k == 12
    res = A[:, idr.redund] - A[:, idr.skel] @ idr.T
    assert np.abs(res).max() < 1e-12 * np.abs(A).max()
    # fewer rows than n + oversample: no sketch, the deterministic ID itself
    B = rng.standard_normal((30, 20))
    r1, r2 = randomized_id(B, 1e-9, 1, 2, 16), cpqr_id(B, 1e-9)
    assert r1.k == r2.k and np.array_equal(r1.skel, r2.skel) and np.array_equal(r1.T, r2.T)


def test_randomized_id_error_on_kernel_blocks():
    # On proxy compression blocks of the star curve the sketched ID reproduces the
    # redundant columns to the precision of the deterministic one (a small factor):
    # |M(:, r) - M(:, s) T| <= 10 max(|R_kk| of the deterministic ID, eps |R_00|).
    import workloads as W
    from oracle import Problem, factor
    from oracle.interp import randomized_id
    from oracle.rs import compression_block
    g = W.star_curve(2048)
    p = Problem("lap2d_sl", g.points, g.weights)
    F = factor(p, 1e-9, 64, 64)
    checked = 0
    for b, r in list(F.records.items())[::7]:
        t = F.tree
        M = compression_block(F.prob, r.J, r.near, t.center[b], 1.5 * t.side[b], 64)
        rid = randomized_id(M, 1e-9, b, 2024, 16)
        if rid.k in (0, M.shape[1]):
            continue
        res = M[:, rid.redund] - M[:, rid.skel] @ rid.T
        bound = 10 * max(r.idr.rdiag[min(r.k, len(r.idr.rdiag) - 1)], 1e-9 * r.idr.rdiag[0])
        assert np.linalg.norm(res, axis=0).max() <= bound, b
        assert abs(rid.k - r.k) <= max(3, r.k // 10), (b, rid.k, r.k)
        checked += 1
    assert checked >= 10
