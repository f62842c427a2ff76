"""Parsimonious bivariate Matern model (paper Section 4.2.1) on the GPU: the
2n x 2n location-major covariance through the same TLR path, against the
dense bivariate oracle.  Bound as for the univariate FP64 path:
|l_TLR - l_dense| <= N max(1e-8, 0.1 tol), N = 2n the matrix size."""
import numpy as np
import pytest

import synthetic
from oracle import bivariate as BV
from oracle import ordering as OO
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


def problem(m, theta, kind="hilbert", extra=0):
    locs = synthetic.jittered_grid(m, synthetic.seed_for(9, synthetic.SEED_LOCS, extra))
    n = locs.shape[0]
    e = synthetic.standard_normal(2 * n, synthetic.seed_for(9, synthetic.SEED_Z, extra))
    z = BV.sample(locs, theta, e).reshape(n, 2)
    perm = OO.reorder(locs, kind)
    return locs[perm], z[perm].reshape(-1)


@pytest.mark.parametrize("m,nb,theta,kind", [
    (20, 100, (1.0, 1.0, 0.1, 0.5, 0.5, 0.5), "hilbert"),      # closed forms for all three functions
    (20, 160, (1.3, 0.7, 0.08, 0.5, 1.5, -0.6), "morton"),     # nu_12 = 1: general-nu tables
    (30, 300, (0.9, 1.6, 0.05, 1.0, 2.5, 0.9), "kdtree"),      # general nu_11, nu_12 = 1.75, ragged last tile
    (30, 256, (1.0, 1.0, 0.1, 1.5, 1.5, 0.0), "hilbert"),      # independent components
    (40, 400, (1.0, 2.0, 0.03, 0.5, 1.5, 0.95), "hilbert"),    # near the validity boundary
])
def test_bivariate_loglik_against_oracle(m, nb, theta, kind):
    device()
    tol = 1e-9
    locs, z = problem(m, theta, kind)
    N = z.size
    # tiles above rank nb/2 are kept dense: smooth, long-range fields on a few
    # hundred locations have near neighbours of high rank
    plan = B.Plan(N, nb, maxrank=nb // 2, dense_tiles=True)
    ws = plan.workspace()
    out = plan.loglik_bivariate(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    ref = BV.loglik(locs, z, theta)
    err = abs(out[2] - ref.loglik)
    print(f"bivariate N={N} nb={nb} theta={theta} {kind}: gpu {out[2]!r} dense {ref.loglik!r} |dl|={err:.2e} "
          f"|dlogdet|={abs(out[0] - ref.logdet):.2e}", flush=True)
    assert plan.status(ws)["code"] == 0, plan.status(ws)
    assert err <= N * max(1e-8, 0.1 * tol)
    assert abs(out[0] - ref.logdet) <= N * max(1e-8, 0.1 * tol)


def test_bivariate_tiles_against_oracle():
    """Compressed off-diagonal tiles of the bivariate covariance (read back
    as U V^T after compression at 1e-13), entry by entry, against the
    oracle's matrix: covers the three functions and the interleaving."""
    device()
    theta = (1.3, 0.7, 0.08, 0.5, 1.5, -0.6)
    locs, z = problem(20, theta, "hilbert", extra=1)
    N, nb = z.size, 160
    sig = BV.covariance_matrix(locs, theta)
    plan2 = B.Plan(N, nb, maxrank=nb)
    ws2 = plan2.workspace()
    dlocs = to_dev(locs)  # kept alive until the stream has run
    B._check(B.lib().tlr_gen_tiles_bivariate(plan2._h, B._ptr(dlocs), B._ThetaBiv(*theta), B._ptr(ws2), ws2.numel(),
                                             B._stream()), "tlr_gen_tiles_bivariate")
    plan2.compress(ws2, 1e-13)
    for (i, j) in [(1, 0), (4, 2), (4, 0)]:
        t, r = plan2.tile(ws2, i, j)
        ref = sig[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
        assert np.max(np.abs(t - ref)) <= 1e-12 * np.max(np.abs(sig)), (i, j, r)


def test_bivariate_rejects_invalid():
    device()
    plan = B.Plan(801, 100)  # odd matrix size
    ws = plan.workspace()
    locs = to_dev(np.full((400, 2), 0.5))
    with pytest.raises(RuntimeError):
        plan.loglik_bivariate(ws, locs, to_dev(np.zeros(801)), (1.0, 1.0, 0.1, 0.5, 0.5, 0.5), 1e-9)
    plan = B.Plan(800, 100)
    ws = plan.workspace()
    with pytest.raises(RuntimeError):
        plan.loglik_bivariate(ws, locs, to_dev(np.zeros(800)), (1.0, 1.0, 0.1, 0.5, 0.5, 1.2), 1e-9)


@pytest.mark.parametrize("m,nb,theta,kind", [
    (30, 300, (1.3, 0.7, 0.08, 0.5, 1.5, -0.6), "hilbert"),
    (40, 400, (1.0, 2.0, 0.03, 0.5, 1.5, 0.95), "morton"),
])
def test_bivariate_mixed_precision(m, nb, theta, kind):
    """A mixed plan (float32 factors) on the bivariate matrix: within the
    mixed bound 1e-6 N of the dense oracle, no rank above the float64 plan's.
    A mixed plan keeps no tile dense, so both plans take the rank cap nb."""
    device()
    tol = 1e-9
    locs, z = problem(m, theta, kind, extra=2)
    N = z.size
    ref = BV.loglik(locs, z, theta)
    outs = {}
    for prec in ("fp64", "mixed_fp32"):
        plan = B.Plan(N, nb, maxrank=nb, precision=prec)
        ws = plan.workspace()
        out = plan.loglik_bivariate(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
        outs[prec] = (out, plan.status(ws))
    (o64, s64), (o32, s32) = outs["fp64"], outs["mixed_fp32"]
    err = abs(o32[2] - ref.loglik)
    print(f"bivariate mixed N={N} nb={nb}: mixed {o32[2]!r} fp64 {o64[2]!r} dense {ref.loglik!r} |dl|/N {err / N:.2e} "
          f"rank sums {s32['rank_sum']} / {s64['rank_sum']}", flush=True)
    assert s32["code"] == 0 and s64["code"] == 0
    assert err <= 1e-6 * N
    assert s32["rank_sum"] <= s64["rank_sum"]
