"""Pins of the oracle parts that the structural tests do not fix by themselves:
the kernel functions (known values and positive definiteness), the norm
estimate nu and the absolute threshold delta of Sec. III-B (closed forms and a
statistical bound from the Gaussian sketch), and the power-method 2-norm of
Sec. V-A (against LAPACK's exact 2-norm).

Expected values are written out as numbers fixed by the formulas of Sec. V-A
(eq. (cov), eq. (ie)) or by the mathematics, never re-derived with the
oracle's own code."""
import math

import numpy as np
import pytest

from oracle.build import _Builder, absolute_threshold
from oracle.h2 import power_method_error
from oracle.kernels import KernelOperator, kernel_from_distance, pair_distance
from oracle.philox import gaussian
from paper_2506_16759_amd.workloads import uniform_points

E_M1 = 0.36787944117144233     # e^-1
E_M2 = 0.1353352832366127      # e^-2
E_MHALF = 0.6065306597126334   # e^-1/2
COS3 = -0.9899924966004454     # cos(3)


# ----------------------------------------------------------------- kernels

def test_exponential_kernel_known_values():
    # eq. (cov): exp(-r/l); at r = l it is 1/e, at r = 2l 1/e^2, at r = 0 one
    r = np.array([0.0, 0.2, 0.4])
    np.testing.assert_allclose(kernel_from_distance("exp", 0.2, r), [1.0, E_M1, E_M2], rtol=1e-15)


def test_gaussian_kernel_known_values():
    # reading: exp(-r^2/(2 l^2)); r = l gives e^-1/2, r = 2l gives e^-2
    r = np.array([0.0, 0.3, 0.6])
    np.testing.assert_allclose(kernel_from_distance("gauss", 0.3, r), [1.0, E_MHALF, E_M2], rtol=1e-15)


def test_helmholtz_kernel_known_values():
    # eq. (ie) with k = 3: cos(3r)/r; zero at 3r = pi/2, -3/pi at 3r = pi,
    # cos(3) at r = 1; reading: 0 on the diagonal (r = 0)
    r = np.array([0.0, math.pi / 6, math.pi / 3, 1.0])
    got = kernel_from_distance("helmholtz", 3.0, r)
    assert got[0] == 0.0
    assert abs(got[1]) < 1e-15
    np.testing.assert_allclose(got[2:], [-3.0 / math.pi, COS3], rtol=1e-15)


def test_distance_and_operator_entries():
    # a 3-4-5 triangle: |x - y| = 5 exactly, so exp(-r/5) = 1/e
    pts = np.array([[0.0, 3.0, 0.0], [0.0, 4.0, 0.0], [0.0, 0.0, 5.0]])
    r = pair_distance(pts, pts)
    np.testing.assert_array_equal(r, [[0, 5, 5], [5, 0, math.sqrt(50)], [5, math.sqrt(50), 0]])
    K = KernelOperator(pts, "exp", 5.0).dense()
    np.testing.assert_allclose(K[0], [1.0, E_M1, E_M1], rtol=1e-15)
    H = KernelOperator(pts, "helmholtz", 3.0).dense()
    assert np.all(np.diag(H) == 0.0)
    np.testing.assert_allclose(H[0, 1], math.cos(15.0) / 5.0, rtol=1e-15)


@pytest.mark.parametrize("kind,param", [("exp", 0.2), ("gauss", 0.1)])
def test_covariance_matrices_are_positive_definite(kind, param):
    # both covariance kernels are positive definite functions (Bochner), so
    # K on distinct points is SPD; a sign or scale slip in the exponent breaks it
    pts = uniform_points(300, 3, 5)
    K = KernelOperator(pts, kind, param).dense()
    np.testing.assert_array_equal(K, K.T)
    assert np.linalg.eigvalsh(K).min() > 0.0


def test_helmholtz_matrix_is_symmetric_with_zero_diagonal():
    pts = uniform_points(200, 3, 6)
    H = KernelOperator(pts, "helmholtz", 3.0).dense()
    np.testing.assert_array_equal(H, H.T)
    assert np.all(np.diag(H) == 0.0)
    # off the diagonal it is cos(3r)/r: |H| <= 1/r
    r = pair_distance(pts, pts)
    off = ~np.eye(200, dtype=bool)
    assert np.all(np.abs(H[off]) <= 1.0 / r[off] * (1 + 1e-15))


# -------------------------------------------------------- nu and delta

def test_threshold_closed_forms():
    # Y0 of ones: ||Y0||_F = sqrt(n d0), nu = sqrt(n)
    n, d0 = 1024, 16
    Y0 = np.ones((n, d0))
    assert absolute_threshold(Y0, d0, 1e-6, 64, "literal") == pytest.approx(1e-6 * 32.0, rel=1e-15)
    assert absolute_threshold(Y0, d0, 1e-6, 64, "fro_scaled") == pytest.approx(1e-6 * 32.0 / 8.0, rel=1e-15)
    assert absolute_threshold(Y0, d0, 2e-6, 1, "fro_scaled") == pytest.approx(2e-6 * 32.0, rel=1e-15)


def test_delta_scales_with_the_square_root_of_the_leaf_count():
    # the two norm modes of one build differ by exactly sqrt(#leaves)
    pts = uniform_points(1500, 2, 4)
    op = KernelOperator(pts, "exp", 0.1)
    hf = _Builder(op, pts, 32, 0.7, 1e-6, 16, 8, 1024, 77, "fro_scaled").run()
    hl = _Builder(op, pts, 32, 0.7, 1e-6, 16, 8, 1024, 77, "literal").run()
    D = hf.tree.depth
    assert hl.delta / hf.delta == pytest.approx(math.sqrt(2 ** D), rel=1e-14)


def test_norm_estimate_is_unbiased_for_the_frobenius_norm():
    # E ||K Omega||_F^2 = d ||K||_F^2 for Gaussian Omega; per column the
    # variance of ||K w||^2 is 2 sum sigma^4.  nu^2 = ||K Omega||_F^2 / d0 over
    # 64 independent Omega (seeds) must average to ||K||_F^2 within 5 standard
    # deviations, and every single estimate must lie within 6.
    n, d0 = 600, 32
    pts = uniform_points(n, 3, 8)
    K = KernelOperator(pts, "exp", 0.2).dense()
    s2 = np.linalg.eigvalsh(K) ** 2
    fro2, var1 = s2.sum(), 2.0 * (s2 ** 2).sum() / d0
    nus2 = []
    for seed in range(64):
        Y0 = K @ gaussian(seed, np.arange(n), 0, d0)
        nus2.append(absolute_threshold(Y0, d0, 1.0, 1, "literal") ** 2)
    nus2 = np.array(nus2)
    assert abs(nus2.mean() - fro2) <= 5.0 * math.sqrt(var1 / 64)
    assert np.all(np.abs(nus2 - fro2) <= 6.0 * math.sqrt(var1))


# ------------------------------------------------------- power method

def test_power_method_matches_the_exact_two_norm():
    # symmetric difference with a clear top eigenvalue: 20 iterations reach
    # LAPACK's 2-norm ratio to rounding
    n = 400
    rng = np.random.default_rng(3)
    Q, _ = np.linalg.qr(rng.standard_normal((n, n)))
    lam = np.concatenate([[2e-6], 1e-7 * rng.random(n - 1)])
    E = (Q * lam) @ Q.T
    pts = uniform_points(n, 2, 9)
    K = KernelOperator(pts, "exp", 0.2).dense()
    exact = np.linalg.norm(E, 2) / np.linalg.norm(K, 2)
    got = power_method_error(lambda v: E @ v, lambda v: K @ v, n)
    assert got == pytest.approx(exact, rel=1e-6)


def test_power_method_never_exceeds_the_two_norm():
    # each iterate is the norm of a unit vector's image, a lower bound of the
    # 2-norm; with the identity as reference the estimate is that of ||K_H - K||_2
    # alone, which on an H^2 error matrix gets within a factor 2 in 20 steps
    from oracle.build import build_h2
    pts = uniform_points(1200, 2, 12)
    op = KernelOperator(pts, "exp", 0.1)
    h = build_h2(op, pts, leaf_size=32, eta=0.7, tol=1e-5, d0=16, d_inc=8, seed=4)
    K = op.dense()
    E = h.dense() - K
    exact = np.linalg.norm(E, 2)
    got = power_method_error(lambda v: E @ v, lambda v: v, pts.shape[1])
    assert 0.5 * exact <= got <= exact * (1 + 1e-12)
    # and the reference factor alone: the estimate of ||K||_2 from below
    kref = power_method_error(lambda v: K @ v, lambda v: v, pts.shape[1])
    assert kref <= np.linalg.norm(K, 2) * (1 + 1e-12)
