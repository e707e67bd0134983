"""Pins of the oracle's QR, column-pivoted QR and interpolative decomposition (Sec. II-B)."""
import numpy as np
import pytest
import scipy.linalg as sla

from oracle.linalg import back_substitute, column_id, cpqr, qr_r_diag, row_id


@pytest.mark.parametrize("m,d", [(10, 6), (64, 32), (40, 40), (20, 33), (1, 5), (7, 1)])
def test_qr_diag_matches_lapack(m, d):
    A = np.random.default_rng(m * 100 + d).standard_normal((m, d))
    r = np.linalg.qr(A, mode="r")
    np.testing.assert_allclose(qr_r_diag(A), np.abs(np.diag(r)), rtol=1e-12, atol=1e-14)


def test_qr_diag_rank_deficient():
    rng = np.random.default_rng(1)
    A = rng.standard_normal((50, 5)) @ rng.standard_normal((5, 12))   # rank 5
    r = qr_r_diag(A)
    assert r[:5].min() > 1e-3 and r[5:].max() < 1e-12 * r[0]


@pytest.mark.parametrize("rows,cols", [(32, 64), (48, 64), (64, 48), (16, 140), (100, 30)])
def test_cpqr_matches_lapack_geqp3(rows, cols):
    # geqp3 (scipy pivoting=True) chooses the largest remaining norm; on generic
    # matrices there are no ties, so pivots and |R| must agree.
    A = np.random.default_rng(rows + 7 * cols).standard_normal((rows, cols))
    k, piv, R = cpqr(A, 0.0)
    _, R2, P2 = sla.qr(A, pivoting=True, mode="economic")
    assert k == min(rows, cols)
    np.testing.assert_array_equal(piv, P2)
    np.testing.assert_allclose(np.abs(R), np.abs(R2), atol=1e-11)


def test_cpqr_downdating_with_graded_columns():
    # columns of very different scale force the norm-recompute safeguard
    rng = np.random.default_rng(3)
    A = rng.standard_normal((30, 40)) * np.logspace(0, -12, 40)[None, :]
    k, piv, R = cpqr(A, 0.0)
    _, R2, P2 = sla.qr(A, pivoting=True, mode="economic")
    np.testing.assert_array_equal(piv[:20], P2[:20])
    np.testing.assert_allclose(np.abs(np.diag(R))[:20], np.abs(np.diag(R2))[:20], rtol=1e-8)


def test_back_substitute_matches_triangular_solve():
    rng = np.random.default_rng(4)
    R11 = np.triu(rng.standard_normal((12, 12))) + 5 * np.eye(12)
    R12 = rng.standard_normal((12, 7))
    np.testing.assert_allclose(back_substitute(R11, R12), sla.solve_triangular(R11, R12), rtol=1e-12)


def test_column_id_identity_and_residual():
    # ||A - A(:,S) [I T] P^T||_F equals ||R_3||_F (ID equation, Sec. II-B)
    rng = np.random.default_rng(5)
    A = rng.standard_normal((40, 9)) @ rng.standard_normal((9, 70)) + 1e-7 * rng.standard_normal((40, 70))
    delta = 1e-4
    S, T, piv, k = column_id(A, delta)
    assert k == 9
    _, _, R = cpqr(A, 0.0)
    IT = np.hstack([np.eye(k), T])
    approx = np.empty_like(A)
    approx[:, piv] = A[:, S] @ IT
    np.testing.assert_allclose(np.linalg.norm(A - approx), np.linalg.norm(R[k:, k:]), rtol=1e-6)


def test_row_id_exact_identity_rows_and_exact_rank():
    rng = np.random.default_rng(6)
    Y = rng.standard_normal((64, 6)) @ rng.standard_normal((6, 32))     # rank 6 samples
    J, U = row_id(Y, 1e-10 * np.linalg.norm(Y))
    assert len(J) == 6 and U.shape == (64, 6)
    np.testing.assert_array_equal(U[J], np.eye(6))                      # bitwise identity rows
    np.testing.assert_allclose(U @ Y[J], Y, atol=1e-11 * np.abs(Y).max())


def test_interpolation_matrix_is_sign_invariant():
    # T = R11^{-1} R12 does not depend on the Householder sign convention:
    # it solves A(:,S) T = A(:,R) in the least-squares sense with exact rank.
    rng = np.random.default_rng(8)
    A = rng.standard_normal((30, 5)) @ rng.standard_normal((5, 20))
    S, T, piv, k = column_id(A, 1e-9)
    ls = np.linalg.lstsq(A[:, S], A[:, piv[k:]], rcond=None)[0]
    np.testing.assert_allclose(T, ls, atol=1e-9)


def test_truncation_rule_first_small_pivot():
    # singular values 1, 1e-2, ..., 1e-10 (5 columns) -> stop when |R_jj| < delta
    rng = np.random.default_rng(9)
    Q1, _ = np.linalg.qr(rng.standard_normal((20, 6)))
    Q2, _ = np.linalg.qr(rng.standard_normal((6, 6)))
    A = Q1 @ np.diag([1, 1e-2, 1e-4, 1e-6, 1e-8, 1e-10]) @ Q2
    for delta, expect in [(1e-3, 2), (1e-5, 3), (1e-7, 4)]:
        k, piv, R = cpqr(A, delta)
        assert k == expect
        assert abs(R[k - 1, k - 1]) >= delta


def test_zero_and_empty_matrices():
    k, piv, R = cpqr(np.zeros((5, 4)), 1e-12)
    assert k == 0
    J, U = row_id(np.zeros((7, 3)), 1e-12)
    assert len(J) == 0 and U.shape == (7, 0)
