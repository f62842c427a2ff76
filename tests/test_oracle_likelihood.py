"""Pins of the oracle's dense log-likelihood (paper Section 1, eq. loglik)."""
import mpmath
import numpy as np
import pytest

import synthetic
from oracle import likelihood as L
from oracle import matern as M

LOG2PI = np.log(2 * np.pi)


def test_single_point_closed_form():
    for s2, z in [(1.0, 0.3), (2.5, -1.7)]:
        got = L.loglik_dense(np.array([[0.4, 0.4]]), np.array([z]), (s2, 0.1, 0.5)).loglik
        ref = -0.5 * LOG2PI - 0.5 * np.log(s2) - z * z / (2 * s2)
        assert got == pytest.approx(ref, rel=1e-15)


def test_two_points_closed_form():
    locs = np.array([[0.1, 0.2], [0.13, 0.24]])  # distance 0.05
    s2, beta = 1.3, 0.1
    rho = np.exp(-0.05 / beta)
    z1, z2 = 0.7, -0.2
    det = s2 * s2 * (1 - rho * rho)
    quad = (z1 * z1 - 2 * rho * z1 * z2 + z2 * z2) / (s2 * (1 - rho * rho))
    ref = -LOG2PI - 0.5 * np.log(det) - 0.5 * quad
    got = L.loglik_dense(locs, np.array([z1, z2]), (s2, beta, 0.5))
    assert got.loglik == pytest.approx(ref, rel=1e-14)
    assert got.logdet == pytest.approx(np.log(det), rel=1e-14)
    assert got.quad == pytest.approx(quad, rel=1e-14)


def _mp_loglik(locs, z, theta, dps=50):
    with mpmath.workdps(dps):
        n = len(z)
        sigma2, beta, nu = (mpmath.mpf(t) for t in theta)
        A = mpmath.matrix(n, n)
        for i in range(n):
            for j in range(n):
                dx = mpmath.mpf(locs[i, 0]) - mpmath.mpf(locs[j, 0])
                dy = mpmath.mpf(locs[i, 1]) - mpmath.mpf(locs[j, 1])
                x = mpmath.sqrt(dx * dx + dy * dy) / beta
                if x == 0:
                    A[i, j] = sigma2
                else:
                    A[i, j] = sigma2 / (mpmath.gamma(nu) * mpmath.power(2, nu - 1)) * x ** nu * mpmath.besselk(nu, x)
        zz = mpmath.matrix([mpmath.mpf(v) for v in z])
        det = mpmath.det(A)
        sol = mpmath.lu_solve(A, zz)
        quad = sum(zz[k] * sol[k] for k in range(n))
        ll = -mpmath.mpf(n) / 2 * mpmath.log(2 * mpmath.pi) - mpmath.log(det) / 2 - quad / 2
        return float(ll), float(mpmath.log(det)), float(quad)


@pytest.mark.parametrize("n,theta", [(9, (1.0, 0.1, 0.5)), (25, (1.2, 0.2, 1.5)), (36, (0.8, 0.05, 1.0)), (64, (1.0, 0.1, 2.5))])
def test_brute_force_high_precision(n, theta):
    m = int(round(np.sqrt(n)))
    locs = synthetic.jittered_grid(m, 100 + n)
    z = synthetic.standard_normal(n, 200 + n)
    ll, logdet, quad = _mp_loglik(locs, z, theta)
    got = L.loglik_dense(locs, z, theta)
    cond = np.linalg.cond(M.covariance_matrix(locs, theta))
    tol = 1e-15 * cond * 10
    assert got.logdet == pytest.approx(logdet, rel=max(1e-13, tol), abs=1e-10)
    assert got.quad == pytest.approx(quad, rel=max(1e-12, tol))
    assert got.loglik == pytest.approx(ll, rel=max(1e-12, tol))


def _ar1_loglik(t, z, sigma2, beta):
    """Exact l of the 1-D exponential model as a Markov chain."""
    ll = -0.5 * LOG2PI - 0.5 * np.log(sigma2) - z[0] ** 2 / (2 * sigma2)
    for k in range(1, len(t)):
        rho = np.exp(-(t[k] - t[k - 1]) / beta)
        var = sigma2 * (1 - rho * rho)
        r = z[k] - rho * z[k - 1]
        ll += -0.5 * LOG2PI - 0.5 * np.log(var) - r * r / (2 * var)
    return ll


@pytest.mark.parametrize("n", [50, 700])
def test_collinear_exponential_is_ar1(n):
    locs = synthetic.collinear_points(n, 31 + n)
    t = locs[:, 0] * np.sqrt(2.0)  # arc length along the diagonal
    sigma2, beta = 1.4, 0.08
    z = synthetic.standard_normal(n, 5 + n)
    ref = _ar1_loglik(t, z, sigma2, beta)
    got = L.loglik_dense(locs, z, (sigma2, beta, 0.5)).loglik
    # rounding of a dense Cholesky: about n * eps * cond(Sigma) relative
    assert got == pytest.approx(ref, rel=max(1e-12, 2 * n * 2.2e-16 * 100))


def test_permutation_rotation_translation_invariance():
    locs = synthetic.jittered_grid(12, 9) * 0.5 + 0.1
    z = synthetic.standard_normal(144, 10)
    theta = (1.0, 0.07, 1.2)
    ref = L.loglik_dense(locs, z, theta).loglik
    perm = np.random.default_rng(3).permutation(144)
    assert L.loglik_dense(locs[perm], z[perm], theta).loglik == pytest.approx(ref, rel=1e-12)
    c, s = np.cos(0.7), np.sin(0.7)
    rot = (locs - 0.3) @ np.array([[c, -s], [s, c]]).T + 0.3
    assert L.loglik_dense(rot, z, theta).loglik == pytest.approx(ref, rel=1e-10)
    assert L.loglik_dense(locs + 0.17, z, theta).loglik == pytest.approx(ref, rel=1e-10)


def test_sigma2_scaling_identity():
    locs = synthetic.jittered_grid(10, 4)
    z = synthetic.standard_normal(100, 5)
    c = 3.7
    a = L.loglik_dense(locs, np.sqrt(c) * z, (c * 1.1, 0.1, 0.5)).loglik
    b = L.loglik_dense(locs, z, (1.1, 0.1, 0.5)).loglik
    assert a == pytest.approx(b - 0.5 * 100 * np.log(c), rel=1e-12)


def test_profile_variance_maximiser():
    # for fixed (beta, nu) the maximising sigma2 is Z^T R^-1 Z / n, R = Sigma / sigma2
    locs = synthetic.jittered_grid(9, 6)
    z = synthetic.standard_normal(81, 7)
    q1 = L.loglik_dense(locs, z, (1.0, 0.12, 1.5)).quad
    s_hat = q1 / 81
    f = lambda s2: L.loglik_dense(locs, z, (s2, 0.12, 1.5)).loglik  # noqa: E731
    assert f(s_hat) > f(s_hat * 1.01) and f(s_hat) > f(s_hat * 0.99)


def test_not_positive_definite_detected():
    locs = np.array([[0.2, 0.2], [0.2, 0.2], [0.5, 0.6]])  # duplicated location
    with pytest.raises(L.NotPositiveDefinite):
        L.loglik_dense(locs, np.array([1.0, 0.5, 0.1]), (1.0, 0.1, 1.5))
    assert L.loglik_value(locs, np.array([1.0, 0.5, 0.1]), (1.0, 0.1, 1.5)) == -np.inf


def test_identifiable_f():
    assert L.identifiable_f((2.0, 0.1, 0.5)) == pytest.approx(20.0)
    assert L.identifiable_f((1.0, 0.5, 1.5)) == pytest.approx(8.0)


def test_sampled_field_has_target_covariance():
    locs = synthetic.jittered_grid(5, 1)
    theta = (1.0, 0.3, 0.5)
    sig = M.covariance_matrix(locs, theta)
    rng = np.random.default_rng(0)
    draws = np.stack([L.sample_field(locs, theta, rng.standard_normal(25)) for _ in range(4000)])
    emp = draws.T @ draws / 4000
    assert np.max(np.abs(emp - sig)) < 0.1
