"""Storage-precision trial for the low-rank factors (the mixed-precision row of
the hot path): how far l moves when the truncated factors of every
off-diagonal tile (paper Section 2) are held in float32 or in bfloat16.

Sigma~ is built as in the tile-truncated oracle -- each off-diagonal tile
replaced by U S V^T from its exact SVD, singular values > tol kept -- and then
U S and V are rounded to the trial format before the tile is formed again:

* float32: both factors rounded to float32, product in float64;
* bfloat16: both factors rounded to bfloat16 (8 significant bits, round to
  nearest even), product accumulated in float32.

The budget of the mixed path is |l(Sigma~_trial) - l(Sigma~)| <= 1e-6 n.
float32 storage meets it with room to spare; bfloat16 misses it by one to
three orders of magnitude or leaves Sigma~ indefinite, which is why the
library stores float32 factors and has no bfloat16 path.
"""
import numpy as np
import pytest

import synthetic
from oracle import likelihood as OL
from oracle import matern as OM
from oracle import ordering as OO
from oracle import tlr as OT


def to_bf16(x):
    """float64 -> nearest bfloat16 (ties to even), returned as float32: keep the
    top 16 bits of the float32 pattern after adding half an ulp of bfloat16."""
    bits = np.asarray(x, dtype=np.float32).view(np.uint32).astype(np.uint64)
    bits = (bits + 0x7FFF + ((bits >> 16) & 1)) & 0xFFFF0000
    return bits.astype(np.uint32).view(np.float32)


def test_bf16_rounding_rule():
    # exactly representable values stay; halfway cases go to the even neighbour
    assert to_bf16(np.array([1.0, -2.5, 0.0]))[1] == np.float32(-2.5)
    one_ulp = 2.0 ** -7  # spacing of bfloat16 in [1, 2)
    v = to_bf16(np.array([1.0 + one_ulp / 2, 1.0 + 1.5 * one_ulp, 1.0 + 0.49 * one_ulp]))
    np.testing.assert_array_equal(v, np.array([1.0, 1.0 + 2 * one_ulp, 1.0], dtype=np.float32))


def trial_matrices(sigma, nb, tol, modes):
    """Sigma~ in each trial format, from one SVD per tile."""
    n = sigma.shape[0]
    out = {m: np.array(sigma, copy=True) for m in modes}
    for (r0, r1) in OT.tile_bounds(n, nb):
        for (c0, c1) in OT.tile_bounds(n, nb):
            if c0 >= r0:
                continue
            u, s, vt = np.linalg.svd(sigma[r0:r1, c0:c1], full_matrices=False)
            r = OT.numerical_rank(s, tol)
            us, v = u[:, :r] * s[:r], vt[:r].T
            for mode in modes:
                if mode == "fp64":
                    t = us @ v.T
                elif mode == "fp32":
                    t = us.astype(np.float32).astype(np.float64) @ v.astype(np.float32).astype(np.float64).T
                else:
                    t = (to_bf16(us) @ to_bf16(v).T).astype(np.float64)  # float32 accumulation
                out[mode][r0:r1, c0:c1] = t
                out[mode][c0:c1, r0:r1] = t.T
    return out


def ell(sigma, z):
    try:
        return OL.loglik_from_matrix(sigma, z).loglik
    except OL.NotPositiveDefinite:
        return None


@pytest.mark.parametrize("beta", [0.03, 0.1, 0.3])
def test_factor_storage_precision(beta):
    theta, nb, tol = (1.0, beta, 0.5), 200, 1e-7
    locs = synthetic.jittered_grid(40, synthetic.seed_for(1, synthetic.SEED_LOCS))
    n = locs.shape[0]
    z = OL.sample_field(locs, theta, synthetic.standard_normal(n, synthetic.seed_for(1, synthetic.SEED_Z)))
    perm = OO.reorder(locs, "hilbert")
    locs, z = locs[perm], z[perm]
    sigma = OM.covariance_matrix(locs, theta)
    mats = trial_matrices(sigma, nb, tol, ("fp64", "fp32", "bf16"))
    base, l32, l16 = (ell(mats[m], z) for m in ("fp64", "fp32", "bf16"))
    print(f"beta={beta}: |dl|/n float32 {abs(l32 - base) / n:.2e}, bfloat16 "
          f"{'not SPD' if l16 is None else f'{abs(l16 - base) / n:.2e}'}")
    assert base is not None and l32 is not None
    assert abs(l32 - base) <= 1e-7 * n
    assert l16 is None or abs(l16 - base) > 1e-6 * n
