"""Nelder-Mead host driver: convergence on problems with known minimisers,
against SciPy's independent implementation, and a small Matern fit through
the dense oracle (CPU only)."""
import math

import numpy as np
import pytest
from scipy import optimize

import synthetic
from oracle import likelihood as OL
from paper_2402_09356_amd.mle import nelder_mead


def test_quadratic_minimum():
    c = np.array([0.3, -1.2, 2.0])
    A = np.diag([1.0, 4.0, 9.0])
    res = nelder_mead(lambda x: float((x - c) @ A @ (x - c)), np.zeros(3), step=0.5, ftol=1e-14, max_evals=5000)
    assert res.converged
    np.testing.assert_allclose(res.x, c, atol=1e-5)


def test_rosenbrock_matches_scipy():
    def rosen(x):
        return float(100.0 * (x[1] - x[0] ** 2) ** 2 + (1.0 - x[0]) ** 2)

    ours = nelder_mead(rosen, np.array([-1.2, 1.0]), step=0.1, ftol=1e-14, max_evals=5000)
    ref = optimize.minimize(rosen, np.array([-1.2, 1.0]), method="Nelder-Mead",
                            options={"xatol": 1e-10, "fatol": 1e-14, "maxfev": 5000})
    np.testing.assert_allclose(ours.x, [1.0, 1.0], atol=1e-5)
    np.testing.assert_allclose(ours.x, ref.x, atol=1e-5)


def test_infinite_values_are_rejected_points():
    # a wall at x < 0 (like a failed factorisation): the minimiser stays feasible
    def f(x):
        return math.inf if x[0] < 0.0 else float((x[0] - 0.5) ** 2 + x[1] ** 2)

    res = nelder_mead(f, np.array([2.0, 1.0]), step=0.5, ftol=1e-14, max_evals=3000)
    np.testing.assert_allclose(res.x, [0.5, 0.0], atol=1e-5)


def test_evaluation_budget_is_respected():
    calls = []
    res = nelder_mead(lambda x: calls.append(1) or float(np.sum(x ** 2)), np.ones(3), ftol=0.0, max_evals=57)
    assert res.evals == len(calls) and res.evals <= 57 + 3  # a shrink may finish its vertices
    assert not res.converged


def test_matern_fit_through_dense_oracle_recovers_theta():
    """Fit (sigma2, beta) at nu = 1/2 on n = 400 points whose Z is drawn from
    theta_true: the estimate is the grid maximiser of the likelihood (checked
    against a brute-force scan of l around it)."""
    theta_true = (1.0, 0.1, 0.5)
    locs = synthetic.jittered_grid(20, 99)
    z = OL.sample_field(locs, theta_true, synthetic.standard_normal(400, 98))

    def negll(x):
        return -OL.loglik_dense(locs, z, (math.exp(x[0]), math.exp(x[1]), 0.5)).loglik

    res = nelder_mead(negll, np.log([0.5, 0.05]), step=0.1, ftol=1e-9, max_evals=1000)
    assert res.converged
    # no point of a small grid around the estimate is better
    for dx in (-0.01, 0.0, 0.01):
        for dy in (-0.01, 0.0, 0.01):
            assert negll(res.x + np.array([dx, dy])) >= res.f - 1e-7
