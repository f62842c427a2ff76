"""Tukey g-and-h (TGH) random field likelihood (paper Section 4.2.2).

TEST INFRASTRUCTURE ONLY (see the package docstring).

The field is T(s) = xi + omega tau(Z(s)) with Z a standard Gaussian random
field (unit variance, Matern correlation of Section 4.1) and

    tau(z) = g^-1 (exp(g z) - 1) exp(h z^2 / 2)        (g != 0)
    tau(z) = z exp(h z^2 / 2)                          (g = 0, the limit)

For h >= 0, tau is strictly increasing, so T has a density by the change of
variables: with z_i = tau^-1((t_i - xi) / omega),

    l_TGH = l_Gauss(z; theta) - sum_i log(omega tau'(z_i)),

l_Gauss the Gaussian log-likelihood of Section 1 (eq. "loglik") and

    tau'(z) = exp(h z^2/2) (exp(g z) + h z (exp(g z) - 1) / g).

tau^-1 has no closed form: it is taken here by plain bisection on a bracket
grown until it holds the value, halved until it is an exact root or two
adjacent floats (the closer of the two is returned).
A value outside the range of tau (h = 0, g != 0: tau maps onto
(-1/g, inf) or (-inf, -1/g)) has no preimage; its density is zero and the
log-likelihood is -inf.  g = h = 0 gives the Gaussian field with mean xi and
covariance omega^2 Sigma.
"""
from __future__ import annotations

import numpy as np

from . import likelihood


def tau(z, g: float, h: float):
    z = np.asarray(z, dtype=np.float64)
    core = z if g == 0.0 else np.expm1(g * z) / g
    return core * np.exp(0.5 * h * z * z)


def tau_prime(z, g: float, h: float):
    z = np.asarray(z, dtype=np.float64)
    core = z if g == 0.0 else np.expm1(g * z) / g
    return np.exp(0.5 * h * z * z) * (np.exp(g * z) + h * z * core)


def tau_inverse(y, g: float, h: float, halvings: int = 2400):
    """z with tau(z) = y, elementwise, by bisection; NaN where y has no preimage."""
    if h < 0.0:
        raise ValueError("h must be >= 0 (tau is then increasing)")
    y = np.asarray(y, dtype=np.float64)
    out = np.full(y.shape, np.nan)
    ok = np.isfinite(y)
    if h == 0.0 and g != 0.0:
        ok &= (g * y > -1.0)  # the range of (exp(g z) - 1)/g is g y > -1
    yy = y[ok]
    lo = -np.ones_like(yy)
    hi = np.ones_like(yy)
    for _ in range(2000):  # grow the bracket until tau(lo) <= y <= tau(hi)
        need_lo = tau(lo, g, h) > yy
        need_hi = tau(hi, g, h) < yy
        if not (need_lo.any() or need_hi.any()):
            break
        lo = np.where(need_lo, 2.0 * lo, lo)
        hi = np.where(need_hi, 2.0 * hi, hi)
    # halve until every bracket is an exact root or two adjacent floats
    for _ in range(halvings):
        open_ = np.nextafter(lo, hi) < hi
        if not open_.any():
            break
        mid = 0.5 * (lo + hi)
        tm = tau(mid, g, h)
        hit = tm == yy
        up = tm < yy
        lo = np.where(open_ & (up | hit), mid, lo)
        hi = np.where(open_ & (~up | hit), mid, hi)
    out[ok] = np.where(tau(hi, g, h) - yy < yy - tau(lo, g, h), hi, lo)  # the closer end
    return out


def log_jacobian(z, omega: float, g: float, h: float) -> float:
    """sum_i log(omega tau'(z_i)) = log |dT/dZ| summed over the observations."""
    return float(np.sum(np.log(omega * tau_prime(z, g, h))))


def loglik_tgh(locs, t, theta, xi: float, omega: float, g: float, h: float) -> float:
    """l_TGH of observations t at ordered locations locs (dense Cholesky);
    -inf when some t_i has no preimage.  theta = (sigma2, beta, nu) of the
    Gaussian field Z (sigma2 = 1 for the standard field of the paper)."""
    y = (np.asarray(t, dtype=np.float64) - xi) / omega
    z = tau_inverse(y, g, h)
    if not np.all(np.isfinite(z)):
        return -np.inf
    return likelihood.loglik_dense(locs, z, theta).loglik - log_jacobian(z, omega, g, h)


def sample_tgh(z, xi: float, omega: float, g: float, h: float):
    """T = xi + omega tau(Z) from a Gaussian draw Z."""
    return xi + omega * tau(z, g, h)
