"""Pins of the Tukey g-and-h oracle (paper Section 4.2.2) against facts that
do not come from its own formulas: the Gaussian special case through the
Matern covariance with a scaled variance, the closed-form inverse when h = 0,
the normalisation of the one-point density and two published moments of the
g-and-h distribution (Tukey's; h = 0: E tau(Z) = (exp(g^2/2) - 1)/g;
g = 0: E tau(Z)^2 = (1 - 2h)^(-3/2))."""
import math

import numpy as np
import pytest
from scipy import integrate

import synthetic
from oracle import likelihood as OL
from oracle import tgh as OG


def support(xi, omega, g, h, zmax=9.0):
    """The range of T over |Z| <= zmax (outside it P < 1e-18) and
    breakpoints at the images of the integers in between."""
    pts = [xi + omega * float(OG.tau(np.array(k), g, h)) for k in range(-4, 5)]
    lo, hi = (xi + omega * float(OG.tau(np.array(v), g, h)) for v in (-zmax, zmax))
    return lo, hi, pts


def one_point_density(t, xi, omega, g, h):
    locs = np.array([[0.5, 0.5]])
    return math.exp(OG.loglik_tgh(locs, np.array([t]), (1.0, 0.1, 0.5), xi, omega, g, h))


@pytest.mark.parametrize("theta", [(1.0, 0.1, 0.5), (1.0, 0.05, 1.5)])
def test_gaussian_special_case(theta):
    """g = h = 0: T = xi + omega Z is Gaussian with covariance omega^2 Sigma."""
    locs = synthetic.jittered_grid(12, synthetic.seed_for(7, synthetic.SEED_LOCS))
    z = OL.sample_field(locs, theta, synthetic.standard_normal(144, synthetic.seed_for(7, synthetic.SEED_Z)))
    xi, omega = 0.7, 1.9
    t = OG.sample_tgh(z, xi, omega, 0.0, 0.0)
    got = OG.loglik_tgh(locs, t, theta, xi, omega, 0.0, 0.0)
    ref = OL.loglik_dense(locs, t - xi, (omega ** 2 * theta[0], theta[1], theta[2])).loglik
    assert abs(got - ref) <= 1e-9 * abs(ref)


@pytest.mark.parametrize("g", [-0.7, 0.3, 1.2])
def test_closed_form_inverse_when_h_is_zero(g):
    """h = 0: tau(z) = (exp(gz) - 1)/g, so z = log(1 + g y)/g, and values
    with g y <= -1 have no preimage."""
    y = np.linspace(-3.0, 3.0, 61)
    z = OG.tau_inverse(y, g, 0.0)
    inside = g * y > -1.0
    ref = np.log1p(g * y[inside]) / g
    np.testing.assert_allclose(z[inside], ref, rtol=1e-13, atol=1e-14)
    assert np.all(np.isnan(z[~inside]))


@pytest.mark.parametrize("g,h", [(0.5, 0.1), (-0.3, 0.2), (0.0, 0.25), (0.8, 0.0), (0.0, 0.0)])
def test_round_trip(g, h):
    z = synthetic.standard_normal(200, synthetic.seed_for(7, synthetic.SEED_Z, 1)) * 2.0
    y = OG.tau(z, g, h)
    np.testing.assert_allclose(OG.tau_inverse(y, g, h), z, rtol=1e-12, atol=1e-13)


@pytest.mark.parametrize("g,h", [(0.5, 0.1), (-0.3, 0.2), (0.0, 0.25), (0.8, 0.0)])
def test_one_point_density_integrates_to_one(g, h):
    """The change of variables is right only if the density of T integrates
    to one: a missing or wrong Jacobian term fails this."""
    xi, omega = -0.4, 1.3
    lo, hi, pts = support(xi, omega, g, h)
    total, err = integrate.quad(one_point_density, lo, hi, args=(xi, omega, g, h), limit=800,
                                points=pts, epsabs=1e-12, epsrel=1e-11)
    assert abs(total - 1.0) < 1e-7, (total, err)


@pytest.mark.parametrize("g", [0.4, -0.6])
def test_mean_when_h_is_zero(g):
    xi, omega = 0.25, 0.8
    lo, hi, pts = support(xi, omega, g, 0.0)
    mean, _ = integrate.quad(lambda t: t * one_point_density(t, xi, omega, g, 0.0), lo, hi, limit=800,
                             points=pts, epsabs=1e-12, epsrel=1e-11)
    assert abs(mean - (xi + omega * math.expm1(0.5 * g * g) / g)) < 1e-7


@pytest.mark.parametrize("h", [0.05, 0.1])
def test_second_moment_when_g_is_zero(h):
    xi, omega = 0.0, 1.0
    lo, hi, pts = support(xi, omega, 0.0, h, zmax=12.0)
    m2, _ = integrate.quad(lambda t: t * t * one_point_density(t, xi, omega, 0.0, h), lo, hi, limit=800,
                           points=pts, epsabs=1e-12, epsrel=1e-11)
    assert abs(m2 - (1.0 - 2.0 * h) ** -1.5) < 1e-6


def test_no_preimage_gives_minus_infinity():
    locs = np.array([[0.2, 0.3], [0.6, 0.1]])
    # g = 1, h = 0: tau > -1, so (t - xi)/omega = -2 has no preimage
    assert OG.loglik_tgh(locs, np.array([0.0, -2.0]), (1.0, 0.1, 0.5), 0.0, 1.0, 1.0, 0.0) == -np.inf
    with pytest.raises(ValueError):
        OG.tau_inverse(np.array([0.0]), 0.1, -0.1)
