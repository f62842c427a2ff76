"""Parsimonious bivariate Matern model (paper Section 4.2.1, eq. "bivmatern").

TEST INFRASTRUCTURE ONLY (see the package docstring).

Two variables observed at the same n locations in the plane (dimension 2).
theta = (sigma2_11, sigma2_22, a, nu_11, nu_22, beta_12):

    C_vw(d) = rho_vw sigma_vv sigma_ww / (Gamma(nu_vw) 2^(nu_vw - 1)) (d/a)^nu_vw K_nu_vw(d/a),

with one range a, nu_12 = (nu_11 + nu_22)/2, rho_vv = 1 and the colocated
correlation

    rho_12 = beta_12 [Gamma(nu_11 + 1)/Gamma(nu_11)]^(1/2) [Gamma(nu_22 + 1)/Gamma(nu_22)]^(1/2)
             Gamma(nu_12) / Gamma(nu_12 + 1),

Gamma(nu + d/2) at d = 2 being Gamma(nu + 1).  The square roots are those of
the cited definition (Gneiting, Kleiber and Schlather 2010): the model is then
valid exactly for |beta_12| <= 1.  Without them, as the formula is printed,
beta_12 = 1 would put rho_12 above that bound for some smoothness pairs
(nu_11 = 1/2, nu_22 = 5/2: 0.833 against 0.745), an invalid model.  Each
C_vw is the univariate Matern function of ``matern`` with variance
rho_vw sigma_vv sigma_ww.

The 2n x 2n covariance is ordered location-major: entry 2p + v is variable v
(0 or 1) at location p, so the spatial ordering of the locations carries over
to the matrix and its tiles.
"""
from __future__ import annotations

import math

import numpy as np

from . import likelihood, matern


def _check(theta):
    s11, s22, a, n11, n22, b12 = (float(v) for v in theta)
    if not (s11 > 0 and s22 > 0 and a > 0 and n11 > 0 and n22 > 0):
        raise ValueError("variances, range and smoothnesses must be positive")
    if not abs(b12) <= 1.0:
        raise ValueError("|beta_12| <= 1 is required for a valid model")
    return s11, s22, a, n11, n22, b12


def rho12(theta) -> float:
    s11, s22, a, n11, n22, b12 = _check(theta)
    n12 = 0.5 * (n11 + n22)
    lg = math.lgamma
    return b12 * math.exp(0.5 * (lg(n11 + 1.0) - lg(n11)) + 0.5 * (lg(n22 + 1.0) - lg(n22)) + lg(n12) - lg(n12 + 1.0))


def component_theta(theta, v: int, w: int):
    """(variance, range, smoothness) of C_vw as a univariate Matern function;
    the variance of the cross function may be zero or negative."""
    s11, s22, a, n11, n22, b12 = _check(theta)
    if v == w == 0:
        return s11, a, n11
    if v == w == 1:
        return s22, a, n22
    return rho12(theta) * math.sqrt(s11 * s22), a, 0.5 * (n11 + n22)


def cross_cov(d, theta, v: int, w: int) -> np.ndarray:
    scale, a, nu = component_theta(theta, v, w)
    # the univariate function with unit variance, scaled (it needs sigma2 > 0)
    return scale * matern.matern(np.asarray(d, dtype=np.float64), (1.0, a, nu))


def covariance_matrix(locs: np.ndarray, theta) -> np.ndarray:
    """2n x 2n location-major covariance of the bivariate field."""
    locs = np.asarray(locs, dtype=np.float64)
    n = locs.shape[0]
    d = matern.distances(locs, locs)
    out = np.empty((2 * n, 2 * n))
    for v in (0, 1):
        for w in (0, 1):
            out[v::2, w::2] = cross_cov(d, theta, v, w)
    return out


def loglik(locs, z, theta) -> likelihood.LogLik:
    """Gaussian log-likelihood (eq. "loglik") of the 2n location-major
    observations z (z[2p + v] = Z_v(s_p))."""
    return likelihood.loglik_from_matrix(covariance_matrix(locs, theta), z)


def sample(locs, theta, e) -> np.ndarray:
    """Z = L e, L the Cholesky factor of the bivariate covariance."""
    sig = covariance_matrix(locs, theta)
    return np.linalg.cholesky(sig) @ np.asarray(e, dtype=np.float64)
