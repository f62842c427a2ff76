"""Smooth-setting workloads (the paper's small-scale study, Section 5.1.1, and
its smooth variant in the appendix): nu = 1 through the general-nu Matern
tables, beta in {0.025, 0.075, 0.2}, n = 1,600 jittered grid, nb = 320,
tol = 1e-7, Morton / Hilbert / KD-tree orderings (workload 6 of the seeded
generators).  l against the dense oracle within max(n max(1e-8, 0.1 tol),
10 |delta_c|), delta_c = l(Sigma~) - l(Sigma) of the tile-truncated oracle;
and one nu-free fit per ordering whose estimate the oracle scores at least as
high as the true theta (a maximiser's defining property, whatever nu-hat is)."""
import math

import pytest

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from oracle import tlr as OT
from paper_2402_09356_amd import binding as B
from paper_2402_09356_amd import mle
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu

BETAS = (0.025, 0.075, 0.2)


def dataset(beta, rep=0):
    theta = (1.0, beta, 1.0)
    locs = synthetic.jittered_grid(40, synthetic.seed_for(6, synthetic.SEED_LOCS, rep))
    e = synthetic.standard_normal(1600, synthetic.seed_for(6, synthetic.SEED_Z, rep))
    return locs, OL.sample_field(locs, theta, e), theta


@pytest.mark.parametrize("beta", BETAS)
@pytest.mark.parametrize("kind", ["morton", "hilbert", "kdtree"])
def test_smooth_loglik(beta, kind):
    device()
    locs, z, theta = dataset(beta)
    perm = OO.reorder(locs, kind)
    lo, zo = locs[perm], z[perm]
    nb, tol = 320, 1e-7
    plan = B.Plan(1600, nb, maxrank=nb // 2, dense_tiles=True)
    ws = plan.workspace()
    out = plan.loglik(ws, to_dev(lo), to_dev(zo), theta, tol).cpu().numpy()
    dense = OL.loglik_dense(lo, zo, theta).loglik
    comp, _ = OT.compressed_loglik(lo, zo, theta, nb, tol, maxrank=nb // 2)
    bnd = max(1600 * max(1e-8, 0.1 * tol), 10 * abs(comp.loglik - dense))
    print(f"smooth nu=1 beta={beta} {kind}: gpu {out[2]!r} dense {dense!r} |dl| {abs(out[2] - dense):.2e} "
          f"bound {bnd:.2e}", flush=True)
    assert plan.status(ws)["code"] == 0
    assert abs(out[2] - dense) <= bnd


@pytest.mark.parametrize("kind", ["morton", "hilbert", "kdtree"])
def test_smooth_fit_per_ordering(kind):
    device()
    locs, z, theta = dataset(0.075)
    perm = OO.reorder(locs, kind)
    lo, zo = locs[perm], z[perm]
    plan = B.Plan(1600, 320, maxrank=160, dense_tiles=True)
    ws = plan.workspace()
    res = mle.fit(plan, ws, to_dev(lo), to_dev(zo), 1e-7, start=(0.5, 0.05, 1.0), ftol=1e-7, max_evals=600)
    at = OL.loglik_dense(lo, zo, res.theta).loglik
    truth = OL.loglik_dense(lo, zo, theta).loglik
    print(f"smooth fit {kind}: theta-hat {res.theta} l {res.loglik!r} oracle {at!r} at truth {truth!r} "
          f"evals {res.evals} converged {res.converged}", flush=True)
    assert math.isfinite(res.loglik)
    assert abs(res.loglik - at) <= max(1600 * 1e-8, 1e-6 * abs(at))
    assert at >= truth - 1e-3
