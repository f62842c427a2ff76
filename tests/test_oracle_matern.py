"""Pins of the oracle's Matern covariance (paper Section 4.1, eq. maternkernel)."""
import mpmath
import numpy as np
import pytest
from scipy import special

from oracle import matern as M


def _mp_matern(d, sigma2, beta, nu, dps=30):
    with mpmath.workdps(dps):
        x = mpmath.mpf(d) / mpmath.mpf(beta)
        if x == 0:
            return mpmath.mpf(sigma2)
        nu = mpmath.mpf(nu)
        return mpmath.mpf(sigma2) / (mpmath.gamma(nu) * mpmath.power(2, nu - 1)) * x ** nu * mpmath.besselk(nu, x)


def test_exponential_kernel_is_nu_half():
    d = np.linspace(0, 3, 301)
    beta = 0.1
    np.testing.assert_allclose(M.matern(d, (1.0, beta, 0.5)), np.exp(-d / beta), rtol=0, atol=0)
    # the general definition reduces to the same values (K_1/2 is elementary)
    np.testing.assert_allclose(M.matern_general(d, (1.0, beta, 0.5)), np.exp(-d / beta), rtol=4e-15, atol=1e-300)


@pytest.mark.parametrize("nu", [0.5, 1.5, 2.5])
def test_closed_forms_against_general_definition(nu):
    d = np.concatenate([np.geomspace(1e-6, 5.0, 200)])
    theta = (1.7, 0.23, nu)
    np.testing.assert_allclose(M.matern_closed_form(d, theta), M.matern_general(d, theta), rtol=1e-13)


@pytest.mark.parametrize("nu", [0.3, 0.5, 1.0, 1.37, 1.5, 2.5, 3.2])
def test_against_mpmath_high_precision(nu):
    theta = (1.3, 0.11, nu)
    for d in [1e-7, 1e-4, 0.01, 0.05, 0.11, 0.3, 1.0, 2.5, 10.0]:
        ref = float(_mp_matern(d, *theta))
        got = float(M.matern(np.array([d]), theta)[0])
        assert got == pytest.approx(ref, rel=5e-13, abs=1e-300), (nu, d)


def test_variance_at_zero_and_continuity():
    for nu in (0.5, 1.0, 1.5, 2.2):
        theta = (2.5, 0.2, nu)
        assert M.matern(np.array([0.0]), theta)[0] == 2.5
        near = M.matern(np.array([1e-10]), theta)[0]
        assert abs(near - 2.5) < 1e-6


def test_bessel_recurrence_holds_for_used_kv():
    # K_{nu+1}(x) = K_{nu-1}(x) + (2 nu / x) K_nu(x)
    for nu in (0.7, 1.3, 2.0):
        x = np.geomspace(1e-3, 30, 50)
        lhs = special.kv(nu + 1, x)
        rhs = special.kv(nu - 1, x) + 2 * nu / x * special.kv(nu, x)
        np.testing.assert_allclose(lhs, rhs, rtol=1e-12)


def test_monotone_decreasing_in_distance_and_sigma_scaling():
    d = np.linspace(0, 2, 101)
    for nu in (0.5, 1.0, 2.5):
        c = M.matern(d, (1.0, 0.1, nu))
        assert np.all(np.diff(c) <= 0)
        np.testing.assert_allclose(M.matern(d, (3.0, 0.1, nu)), 3.0 * c, rtol=1e-15)


def test_parametrisation_is_d_over_beta_not_sqrt2nu():
    # at d = beta the exponential kernel equals e^-1 exactly as printed
    assert M.matern(np.array([0.25]), (1.0, 0.25, 0.5))[0] == pytest.approx(np.exp(-1.0), rel=1e-16)
    # nu = 3/2 at x = 1: (1 + 1) e^-1, not the sqrt(3)-scaled variant
    assert M.matern(np.array([0.25]), (1.0, 0.25, 1.5))[0] == pytest.approx(2 * np.exp(-1.0), rel=1e-15)


def test_invalid_theta_rejected():
    with pytest.raises(ValueError):
        M.matern(np.array([0.1]), (1.0, -0.1, 0.5))
    with pytest.raises(ValueError):
        M.matern(np.array([0.1]), (np.nan, 0.1, 0.5))


def test_covariance_matrix_symmetric_unit_diagonal():
    rng = np.random.default_rng(0)
    locs = rng.uniform(size=(50, 2))
    s = M.covariance_matrix(locs, (1.0, 0.1, 1.0))
    assert np.array_equal(s, s.T)
    assert np.all(np.diag(s) == 1.0)
