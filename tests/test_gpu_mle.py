"""Nelder-Mead MLE through the GPU library against the same fit through the
dense oracle (C1: n = 1,600 jittered grid, Morton, nb = 200, tol = 1e-9)."""
import math

import numpy as np
import pytest

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from paper_2402_09356_amd import binding as B
from paper_2402_09356_amd import mle
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


def test_fit_matches_dense_oracle_fit():
    device()
    theta_true, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs = synthetic.jittered_grid(40, synthetic.seed_for(1, synthetic.SEED_LOCS))
    e = synthetic.standard_normal(1600, synthetic.seed_for(1, synthetic.SEED_Z))
    z = OL.sample_field(locs, theta_true, e)
    perm = OO.reorder(locs, "morton")
    locs, z = locs[perm], z[perm]
    plan = B.Plan(1600, nb)
    ws = plan.workspace()
    gpu = mle.fit(plan, ws, to_dev(locs), to_dev(z), tol, start=(0.5, 0.05, 1.0), nu=0.5, ftol=1e-9,
                  max_evals=400)
    ref = mle.nelder_mead(lambda x: -OL.loglik_dense(locs, z, (math.exp(x[0]), math.exp(x[1]), 0.5)).loglik,
                          np.log([0.5, 0.05]), step=0.1, ftol=1e-9, max_evals=400)
    ref_theta = (math.exp(ref.x[0]), math.exp(ref.x[1]))
    print("gpu", gpu.theta, gpu.loglik, gpu.evals, "oracle", ref_theta, -ref.f, ref.evals, flush=True)
    assert gpu.converged and ref.converged
    # both sit at the maximiser of nearly the same surface
    assert abs(gpu.theta[0] - ref_theta[0]) <= 1e-3 * ref_theta[0]
    assert abs(gpu.theta[1] - ref_theta[1]) <= 1e-3 * ref_theta[1]
    dense_at_gpu = OL.loglik_dense(locs, z, gpu.theta).loglik
    assert abs(gpu.loglik - dense_at_gpu) <= 1600 * 1e-8 + 1e-6 * abs(dense_at_gpu)
    assert abs(gpu.f_identifiable - gpu.theta[0] * gpu.theta[1] ** -1.0) < 1e-12 * gpu.f_identifiable


def test_nu_free_fit_lands_on_an_oracle_maximiser():
    """All three parameters free from (0.5, 0.05, 1.0), so every simplex move
    of nu goes through the general-nu Matern tables.  The GPU's theta-hat must
    be a local maximiser of the dense oracle's l (every +-1% move in each
    log-parameter lowers it), and the two l agree there within the bound."""
    device()
    theta_true, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs = synthetic.jittered_grid(40, synthetic.seed_for(1, synthetic.SEED_LOCS))
    e = synthetic.standard_normal(1600, synthetic.seed_for(1, synthetic.SEED_Z))
    z = OL.sample_field(locs, theta_true, e)
    perm = OO.reorder(locs, "morton")
    locs, z = locs[perm], z[perm]
    plan = B.Plan(1600, nb)
    ws = plan.workspace()
    gpu = mle.fit(plan, ws, to_dev(locs), to_dev(z), tol, start=(0.5, 0.05, 1.0), ftol=1e-9, max_evals=800)
    at = OL.loglik_dense(locs, z, gpu.theta).loglik
    print("nu-free gpu fit", gpu.theta, gpu.loglik, gpu.evals, "oracle at theta-hat", at, flush=True)
    assert gpu.converged
    assert abs(gpu.loglik - at) <= 1600 * 1e-8
    for i in range(3):
        for sgn in (-1.0, 1.0):
            th = list(gpu.theta)
            th[i] *= math.exp(sgn * 0.01)
            assert OL.loglik_dense(locs, z, tuple(th)).loglik < at, (i, sgn)
