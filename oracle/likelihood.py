"""Dense Gaussian log-likelihood (paper Section 1, eq. "loglik").

    l(theta) = -(n/2) log(2 pi) - (1/2) log|Sigma(theta)| - (1/2) Z^T Sigma^-1 Z

computed through the lower Cholesky factor L of Sigma: log|Sigma| = 2 sum log
L_ii and Z^T Sigma^-1 Z = y^T y with y = L^-1 Z.  A failed Cholesky means
Sigma is not (numerically) positive definite.

Also: the identifiable combination f = sigma2 * beta^(-2 nu) reported beside
parameter estimates (Section 5.1.1, eq. "functionforder").
"""
from __future__ import annotations

from dataclasses import dataclass

import numpy as np
from scipy import linalg

from . import matern

LOG_2PI = float(np.log(2.0 * np.pi))


class NotPositiveDefinite(ArithmeticError):
    pass


@dataclass
class LogLik:
    loglik: float
    logdet: float
    quad: float
    n: int


def loglik_from_matrix(sigma: np.ndarray, z: np.ndarray) -> LogLik:
    """l from an explicit covariance matrix and observation vector."""
    sigma = np.asarray(sigma, dtype=np.float64)
    z = np.asarray(z, dtype=np.float64)
    n = z.size
    try:
        chol = linalg.cholesky(sigma, lower=True, check_finite=True)
    except linalg.LinAlgError as exc:  # not SPD
        raise NotPositiveDefinite(str(exc)) from exc
    diag = np.diag(chol)
    if np.any(diag <= 0) or not np.all(np.isfinite(diag)):
        raise NotPositiveDefinite("non-positive pivot")
    logdet = 2.0 * float(np.sum(np.log(diag)))
    y = linalg.solve_triangular(chol, z, lower=True)
    quad = float(y @ y)
    ll = -0.5 * n * LOG_2PI - 0.5 * logdet - 0.5 * quad
    return LogLik(ll, logdet, quad, n)


def loglik_dense(locs: np.ndarray, z: np.ndarray, theta) -> LogLik:
    """l(theta) for locations and observations in a common order."""
    return loglik_from_matrix(matern.covariance_matrix(locs, theta), z)


def loglik_value(locs, z, theta) -> float:
    """l(theta), or -inf when Sigma(theta) is not positive definite."""
    try:
        return loglik_dense(locs, z, theta).loglik
    except (NotPositiveDefinite, ValueError):
        return -np.inf


def sample_field(locs: np.ndarray, theta, e: np.ndarray) -> np.ndarray:
    """Z = L e with L the lower Cholesky factor of Sigma(theta) (generation order)."""
    sigma = matern.covariance_matrix(locs, theta)
    chol = linalg.cholesky(sigma, lower=True)
    return chol @ np.asarray(e, dtype=np.float64)


def identifiable_f(theta) -> float:
    """f(sigma2, beta, nu) = sigma2 * beta^(-2 nu)."""
    sigma2, beta, nu = (float(t) for t in theta)
    return sigma2 * beta ** (-2.0 * nu)
