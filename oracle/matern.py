"""Univariate Matern covariance and dense covariance assembly.

Definition (paper Section 4.1, eq. "maternkernel"), theta = (sigma2, beta, nu):

    C(d; theta) = sigma2 / (Gamma(nu) 2^(nu-1)) * (d/beta)^nu * K_nu(d/beta),

with d the Euclidean distance, no nugget, and C(0) = sigma2 (the limit as
d -> 0+).  The argument of K_nu is d/beta exactly as printed (no sqrt(2 nu)
rescaling).

For nu = 1/2, 3/2, 5/2, K_nu is elementary and the definition reduces exactly
to sigma2 e^-x, sigma2 (1+x) e^-x and sigma2 (1 + x + x^2/3) e^-x with
x = d/beta; these closed forms are used there.  Any other nu uses SciPy's K_nu
(``scipy.special.kv``) and Gamma.

Covariance assembly (paper eq. "covfunc" and eq. "staconv"):
Sigma_ij = C(||s_i - s_j||; theta).
"""
from __future__ import annotations

import numpy as np
from scipy import special

HALF_INTEGER_NUS = (0.5, 1.5, 2.5)


def _check_theta(theta):
    sigma2, beta, nu = (float(t) for t in theta)
    if not (np.isfinite(sigma2) and np.isfinite(beta) and np.isfinite(nu)):
        raise ValueError("theta must be finite")
    if sigma2 <= 0 or beta <= 0 or nu <= 0:
        raise ValueError("theta components must be positive")
    return sigma2, beta, nu


def matern_general(d, theta) -> np.ndarray:
    """The printed definition with SciPy's K_nu, for any nu > 0."""
    sigma2, beta, nu = _check_theta(theta)
    d = np.asarray(d, dtype=np.float64)
    x = d / beta
    out = np.full(d.shape, sigma2, dtype=np.float64)
    pos = x > 0
    xp = x[pos]
    coef = sigma2 / (special.gamma(nu) * 2.0 ** (nu - 1.0))
    with np.errstate(over="ignore", invalid="ignore", under="ignore"):
        val = coef * xp ** nu * special.kv(nu, xp)
    # K_nu underflows to 0 for very large x; the product is then 0 as well.
    val = np.where(np.isfinite(val), val, 0.0)
    out[pos] = val
    return out


def matern_closed_form(d, theta) -> np.ndarray:
    """Exact elementary forms for nu in {1/2, 3/2, 5/2}."""
    sigma2, beta, nu = _check_theta(theta)
    d = np.asarray(d, dtype=np.float64)
    x = d / beta
    e = np.exp(-x)
    if nu == 0.5:
        return sigma2 * e
    if nu == 1.5:
        return sigma2 * (1.0 + x) * e
    if nu == 2.5:
        return sigma2 * (1.0 + x + x * x / 3.0) * e
    raise ValueError("closed form only for nu in {0.5, 1.5, 2.5}")


def matern(d, theta) -> np.ndarray:
    """C(d; theta): closed form at half-integer nu, SciPy K_nu otherwise."""
    nu = float(theta[2])
    if nu in HALF_INTEGER_NUS:
        return matern_closed_form(d, theta)
    return matern_general(d, theta)


def distances(a: np.ndarray, b: np.ndarray) -> np.ndarray:
    """Euclidean distance matrix between rows of a (m x 2) and b (k x 2)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    dx = a[:, 0][:, None] - b[:, 0][None, :]
    dy = a[:, 1][:, None] - b[:, 1][None, :]
    return np.sqrt(dx * dx + dy * dy)


def covariance(a: np.ndarray, b: np.ndarray, theta) -> np.ndarray:
    """Block of Sigma between point sets a and b."""
    return matern(distances(a, b), theta)


def covariance_matrix(locs: np.ndarray, theta) -> np.ndarray:
    """Full n x n Sigma(theta) for locations in their given order."""
    return covariance(locs, locs, theta)
