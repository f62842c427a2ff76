"""Pins of the blocked dense oracle (used where Sigma does not fit as one array).

Each check compares it with something it shares no code with: LAPACK's
unblocked Cholesky on the whole matrix, the exact Markov factorisation of the
one-dimensional exponential model, and a direct draw Z = L e.
"""
import numpy as np
import pytest
from scipy import linalg

import synthetic
from oracle import blocked as OB
from oracle import likelihood as OL
from oracle import matern as OM

LOG2PI = float(np.log(2 * np.pi))


@pytest.mark.parametrize("theta,b", [((1.0, 0.1, 0.5), 128), ((0.7, 0.05, 1.5), 200), ((1.3, 0.2, 1.0), 700)])
def test_blocked_equals_unblocked(theta, b):
    locs = synthetic.jittered_grid(26, 41)  # n = 676: ragged last block for b = 128, 200
    z = synthetic.standard_normal(676, 42)
    ref = OL.loglik_dense(locs, z, theta)
    got = OB.loglik_blocked(locs, z, theta, b=b)
    assert got.logdet == pytest.approx(ref.logdet, rel=1e-11, abs=1e-9)
    assert got.quad == pytest.approx(ref.quad, rel=1e-10)
    assert got.loglik == pytest.approx(ref.loglik, rel=1e-11)


def _ar1_loglik(t, z, sigma2, beta):
    ll = -0.5 * LOG2PI - 0.5 * np.log(sigma2) - z[0] ** 2 / (2 * sigma2)
    rho = np.exp(-np.diff(t) / beta)
    var = sigma2 * (1 - rho * rho)
    r = z[1:] - rho * z[:-1]
    return ll + float(np.sum(-0.5 * LOG2PI - 0.5 * np.log(var) - r * r / (2 * var)))


def test_blocked_memmap_matches_markov_chain(tmp_path):
    # collinear points with nu = 1/2 form an AR(1) chain: l is exact in O(n)
    n = 2500
    locs = synthetic.collinear_points(n, 77)
    t = locs[:, 0] * np.sqrt(2.0)
    e = synthetic.standard_normal(n, 78)
    sigma2, beta = 0.9, 0.05
    # Z drawn from the chain itself, so that y = L^-1 Z stays of unit size
    rho = np.exp(-np.diff(t) / beta)
    z = np.empty(n)
    z[0] = np.sqrt(sigma2) * e[0]
    for k in range(1, n):
        z[k] = rho[k - 1] * z[k - 1] + np.sqrt(sigma2 * (1 - rho[k - 1] ** 2)) * e[k]
    ref = _ar1_loglik(t, z, sigma2, beta)
    got = OB.loglik_blocked(locs, z, (sigma2, beta, 0.5), b=512, path=str(tmp_path / "blocks.bin"))
    assert got.loglik == pytest.approx(ref, rel=1e-10)
    assert not (tmp_path / "blocks.bin").exists()


def test_matvec_draws_with_the_factor():
    locs = synthetic.jittered_grid(15, 5)
    theta = (1.0, 0.15, 0.5)
    e = synthetic.standard_normal(225, 6)
    f = OB.BlockedCholesky(locs, theta, b=64)
    chol = linalg.cholesky(OM.covariance_matrix(locs, theta), lower=True)
    np.testing.assert_allclose(f.matvec(e), chol @ e, rtol=1e-11, atol=1e-12)
    # with Z = L e, y = L^-1 Z recovers e and quad = e^T e
    res = f.loglik(chol @ e)
    assert res.quad == pytest.approx(float(e @ e), rel=1e-9)
    f.close()


def test_blocked_not_positive_definite():
    locs = np.array([[0.2, 0.2], [0.2, 0.2], [0.5, 0.6], [0.1, 0.9]])  # duplicated location
    with pytest.raises(OL.NotPositiveDefinite):
        OB.loglik_blocked(locs, np.ones(4), (1.0, 0.1, 1.5), b=2)


@pytest.mark.parametrize("nb,tol", [(100, 1e-5), (150, 1e-7)])
def test_tile_truncated_blocked_equals_compressed_matrix(nb, tol):
    # the tile-truncated covariance assembled block by block gives the same l
    # as the whole-matrix construction of the tile oracle
    from oracle import tlr as OT

    locs = synthetic.jittered_grid(24, 51)  # n = 576
    z = synthetic.standard_normal(576, 52)
    theta = (1.0, 0.15, 1.5)
    ref, _ = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=nb)
    got = OB.loglik_blocked(locs, z, theta, b=3 * nb, tiles=(nb, tol, nb))
    assert got.loglik == pytest.approx(ref.loglik, rel=1e-10, abs=1e-8)
    exact = OL.loglik_dense(locs, z, theta).loglik
    assert abs(got.loglik - exact) > 0  # truncation did change the matrix
