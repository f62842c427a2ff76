"""Pins of the bivariate Matern oracle (paper Section 4.2.1, eq. "bivmatern")
against facts outside its own formulas:

* beta_12 = 0: the two variables are independent, so l is the sum of two
  univariate likelihoods of the interleaved halves;
* nu_11 = nu_22: the model is separable, Sigma = C (x) B (Kronecker product of
  the location correlation and the 2 x 2 colocated covariance), whose
  log-determinant and quadratic form have closed forms in C and B;
* validity: the colocated-correlation normalisation puts beta_12 = 1 exactly
  on the boundary of positive definiteness: the matrix is positive definite
  there and indefinite 2% beyond (brute-force eigenvalues), which pins the
  square roots of the cited definition (the printed form, without them, is
  indefinite at beta_12 = 1 for nu = 1/2, 5/2).
"""
import numpy as np
import pytest
from scipy import linalg

import synthetic
from oracle import bivariate as BV
from oracle import likelihood as OL
from oracle import matern as OM


def grid(m, extra=0):
    return synthetic.jittered_grid(m, synthetic.seed_for(9, synthetic.SEED_LOCS, extra))


def draw(locs, theta, extra=0):
    e = synthetic.standard_normal(2 * locs.shape[0], synthetic.seed_for(9, synthetic.SEED_Z, extra))
    return BV.sample(locs, theta, e)


def test_independent_components():
    locs = grid(15)
    theta = (1.3, 0.7, 0.08, 0.5, 1.5, 0.0)
    z = draw(locs, (1.3, 0.7, 0.08, 0.5, 1.5, 0.4))
    got = BV.loglik(locs, z, theta).loglik
    ref = (OL.loglik_dense(locs, z[0::2], (1.3, 0.08, 0.5)).loglik +
           OL.loglik_dense(locs, z[1::2], (0.7, 0.08, 1.5)).loglik)
    assert abs(got - ref) <= 1e-10 * abs(ref)


@pytest.mark.parametrize("nu,beta12", [(0.5, 0.6), (1.5, -0.35), (1.0, 0.9)])
def test_separable_case_closed_form(nu, beta12):
    locs = grid(14, 1)
    n = locs.shape[0]
    s11, s22, a = 1.4, 0.6, 0.1
    theta = (s11, s22, a, nu, nu, beta12)
    z = draw(locs, theta, 1)
    # Sigma = C (x) B, C the unit-variance Matern correlation of the locations,
    # B the colocated covariance (rho_12 = beta_12 when the smoothnesses agree)
    C = OM.covariance_matrix(locs, (1.0, a, nu))
    B = np.array([[s11, beta12 * np.sqrt(s11 * s22)], [beta12 * np.sqrt(s11 * s22), s22]])
    cf = linalg.cho_factor(C, lower=True)
    logdet = 2.0 * (2.0 * np.sum(np.log(np.diag(cf[0])))) + n * np.log(np.linalg.det(B))
    Zm = z.reshape(n, 2)  # row p = (Z_0(s_p), Z_1(s_p))
    quad = float(np.trace(np.linalg.solve(B, Zm.T @ linalg.cho_solve(cf, Zm))))
    ref = -0.5 * 2 * n * OL.LOG_2PI - 0.5 * logdet - 0.5 * quad
    got = BV.loglik(locs, z, theta)
    assert abs(got.logdet - logdet) <= 1e-9 * abs(logdet)
    assert abs(got.quad - quad) <= 1e-9 * abs(quad)
    assert abs(got.loglik - ref) <= 1e-9 * abs(ref)


def _min_eig_with_rho(locs, a, n11, n22, rho):
    d = OM.distances(locs, locs)
    n = locs.shape[0]
    out = np.empty((2 * n, 2 * n))
    out[0::2, 0::2] = OM.matern(d, (1.0, a, n11))
    out[1::2, 1::2] = OM.matern(d, (1.0, a, n22))
    out[0::2, 1::2] = rho * OM.matern(d, (1.0, a, 0.5 * (n11 + n22)))
    out[1::2, 0::2] = out[0::2, 1::2].T
    return np.linalg.eigvalsh(out)[0]


@pytest.mark.parametrize("n11,n22", [(0.5, 2.5), (0.5, 1.5), (1.0, 2.0)])
def test_beta_one_is_the_validity_boundary(n11, n22):
    locs = grid(20, 2)
    a = 0.1
    theta = (1.0, 1.0, a, n11, n22, 1.0)
    assert np.linalg.eigvalsh(BV.covariance_matrix(locs, theta))[0] > 0.0
    r1 = BV.rho12(theta)
    assert _min_eig_with_rho(locs, a, n11, n22, 1.02 * r1) < -1e-3
    if (n11, n22) == (0.5, 2.5):
        # the formula as printed, without the square roots
        printed = n11 * n22 / (0.5 * (n11 + n22))
        assert printed > 1.1 * r1 and _min_eig_with_rho(locs, a, n11, n22, printed) < -1.0


def test_invalid_parameters_rejected():
    with pytest.raises(ValueError):
        BV.rho12((1.0, 1.0, 0.1, 0.5, 1.5, 1.01))
    with pytest.raises(ValueError):
        BV.rho12((1.0, 0.0, 0.1, 0.5, 1.5, 0.5))
