"""Pins of the oracle's two-sided construction and of the H^2 low-rank update.

* Special case: for a symmetric matrix and Omega' = Omega the two-sided
  construction must reproduce the symmetric one exactly.
* Closed form: A = Phi Psi^T (non-symmetric, rank r) is recovered exactly, with
  ranks <= r at every cluster of both sides -- a near or far subtraction that
  uses the wrong block, side or transpose leaves a residual and raises ranks.
* Accuracy bound against the dense matrix for A = K + U V^T.
* H^2 entries (plain definition of the format) against columns of the matvec,
  which is computed by up/downsweeps and never forms a basis.
* Transposed matvec against the dense reconstruction.
"""
import numpy as np
import pytest

from oracle.build import build_h2
from oracle.kernels import CallbackOperator, KernelOperator
from oracle.update import LowRankUpdateOperator, build_h2_two_sided, update_h2
from paper_2506_16759_amd.workloads import uniform_points


def _dense_op(A):
    return CallbackOperator(A.shape[0], lambda x: A @ x, lambda r, c: A[np.ix_(r, c)],
                            sketch_t=lambda x: A.T @ x, symmetric=False)


@pytest.fixture(scope="module")
def small():
    pts = uniform_points(1500, 2, 5)
    op = KernelOperator(pts, "exp", 0.2)
    return pts, op, op.dense()


def test_two_sided_reduces_to_symmetric_build(small):
    pts, op, _ = small
    hs = build_h2(op, pts, 32, 0.7, 1e-7, 16, 8, 1024, 11)
    h2 = build_h2_two_sided(op, pts, 32, 0.7, 1e-7, 16, 8, 1024, 11, seed_c=11)
    assert hs.samples == h2.samples and hs.top == h2.top
    for key, sk in hs.skel.items():
        np.testing.assert_array_equal(sk, h2.skel[key])
        np.testing.assert_array_equal(sk, h2.skel_c[key])
    for i, u in hs.U.items():
        np.testing.assert_array_equal(u, h2.U[i])
        np.testing.assert_array_equal(u, h2.Uc[i])
    for key, e in hs.E.items():
        np.testing.assert_array_equal(e, h2.E[key])
        np.testing.assert_array_equal(e, h2.Ec[key])
    for key, b in hs.B.items():
        np.testing.assert_array_equal(b, h2.B[key])


@pytest.mark.parametrize("dim,r", [(2, 6), (3, 12)])
def test_two_sided_exact_low_rank(dim, r):
    n = 1200
    pts = uniform_points(n, dim, 20 + r)
    rng = np.random.default_rng(r)
    Phi, Psi = rng.standard_normal((n, r)), rng.standard_normal((n, r))
    A = Phi @ Psi.T
    h = build_h2_two_sided(_dense_op(A), pts, 32, 0.7, 1e-13, 16, 8, 64, 3)
    for t, ks in h.ranks().items():
        assert ks.max() <= r
        kc = np.array([h.rank_c(t, i) for i in range(1 << t)])
        assert kc.max() <= r
    assert np.linalg.norm(A - h.dense()) / np.linalg.norm(A) <= 1e-12


def test_two_sided_nonsymmetric_accuracy(small):
    pts, _, K = small
    n = K.shape[0]
    rng = np.random.default_rng(3)
    U, V = rng.standard_normal((n, 8)) / np.sqrt(n), rng.standard_normal((n, 8)) / np.sqrt(n)
    A = K + 5.0 * U @ V.T
    tol = 1e-7
    h = build_h2_two_sided(_dense_op(A), pts, 32, 0.7, tol, 16, 8, 1024, 11)
    assert h.two_sided
    Ah = h.dense()
    assert np.linalg.norm(A - Ah) / np.linalg.norm(A) <= 10 * tol
    x = rng.standard_normal((n, 3))
    np.testing.assert_allclose(h.matvec(x), Ah @ x, rtol=0, atol=1e-12 * np.abs(Ah @ x).max())
    np.testing.assert_allclose(h.matvec_t(x), Ah.T @ x, rtol=0, atol=1e-12 * np.abs(Ah.T @ x).max())


def test_entries_match_matvec_columns(small):
    pts, op, _ = small
    n = pts.shape[1]
    hs = build_h2(op, pts, 32, 0.7, 1e-6, 16, 8, 1024, 11)
    rng = np.random.default_rng(0)
    rows = rng.choice(n, 300, replace=False)
    cols = rng.choice(n, 40, replace=False)
    E = np.zeros((n, cols.size))
    E[cols, np.arange(cols.size)] = 1.0
    ref = hs.matvec(E)[rows]
    got = hs.entries(rows, cols)
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13)
    # and for a two-sided matrix
    U = rng.standard_normal((n, 4)) / np.sqrt(n)
    h2 = build_h2_two_sided(LowRankUpdateOperator(hs, U, 2 * U[::-1]), pts, 32, 0.7, 1e-6, 16, 8, 1024, 5)
    np.testing.assert_allclose(h2.entries(rows, cols), h2.matvec(E)[rows], rtol=0, atol=1e-13)


def test_update_of_h2_matrix(small):
    pts, op, _ = small
    n = pts.shape[1]
    tol = 1e-7
    hs = build_h2(op, pts, 32, 0.7, tol, 16, 8, 1024, 11)
    rng = np.random.default_rng(9)
    # update comparable in norm to the matrix itself
    U, V = 100 * rng.standard_normal((n, 16)) / np.sqrt(n), rng.standard_normal((n, 16)) / np.sqrt(n)
    op_u = LowRankUpdateOperator(hs, U, V)
    A = hs.dense() + U @ V.T
    x = rng.standard_normal((n, 2))
    np.testing.assert_allclose(op_u.sketch(x), A @ x, rtol=0, atol=1e-12 * np.abs(A @ x).max())
    np.testing.assert_allclose(op_u.sketch_t(x), A.T @ x, rtol=0, atol=1e-12 * np.abs(A.T @ x).max())
    hu = update_h2(hs, pts, U, V, 32, 0.7, tol, 16, 8)
    assert np.linalg.norm(A - hu.dense()) / np.linalg.norm(A) <= 10 * tol
    # the update keeps the partition
    np.testing.assert_array_equal(hu.tree.perm, hs.tree.perm)
    with pytest.raises(ValueError):
        update_h2(hs, pts, U, V, 16, 0.7, tol, 16, 8)


def test_update_with_full_rank_leaves_meets_tolerance():
    """A rank-64 update makes every 64-point leaf block row full rank: the
    convergence test must keep an oversampling margin, or nearly square
    Gaussian sketches truncate such blocks (error ~70 tol without the margin)."""
    from paper_2506_16759_amd.workloads import gaussian_factors
    n, tol = 4096, 1e-6
    pts = uniform_points(n, 3, 2)
    op = KernelOperator(pts, "exp", 0.2)
    h = build_h2(op, pts, 64, 0.7, tol, 32, 16, 256, 1001)
    U, V = gaussian_factors(n, 64, 3)
    hu = update_h2(h, pts, U, V, 64, 0.7, tol, 32, 16, 256, 1002, oversample=5)
    A = h.dense() + U @ V.T
    assert np.linalg.norm(A - hu.dense()) / np.linalg.norm(A) <= 10 * tol
    # without the margin the full-rank leaves are truncated
    hu0 = update_h2(h, pts, U, V, 64, 0.7, tol, 32, 16, 256, 1002, oversample=0)
    assert np.linalg.norm(A - hu0.dense()) / np.linalg.norm(A) > 10 * tol
