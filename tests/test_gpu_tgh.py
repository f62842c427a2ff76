"""Tukey g-and-h random fields (paper Section 4.2.2) on the GPU against the
oracle: the inverse transform elementwise, and the change-of-variables
log-likelihood on top of the TLR Gaussian one.

Bounds: the inverse to 1e-12 relative (Newton to a few ulps on the device,
bisection to float64 resolution in the oracle); l_TGH within the FP64 TLR
bound n max(1e-8, 0.1 tol) of the dense oracle (the Jacobian sum adds only
rounding)."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from oracle import tgh as OG
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu

PARAMS = [(0.5, 0.1), (-0.3, 0.2), (0.0, 0.25), (0.8, 0.0), (-1.2, 0.0), (0.0, 0.0), (1.5, 0.5)]


@pytest.mark.parametrize("g,h", PARAMS)
def test_inverse_against_oracle(g, h):
    device()
    n = 4096 + 37  # ragged against the 256-thread blocks
    z = 2.5 * synthetic.standard_normal(n, synthetic.seed_for(8, synthetic.SEED_Z))
    xi, omega = 0.3, 1.7
    t = OG.sample_tgh(z, xi, omega, g, h)
    t[:4] = [xi, xi + 1e-13, xi - 1e-12, xi + 5.0]
    if h == 0.0 and g != 0.0:
        t[4] = xi - 2.0 * omega / g  # below (g > 0) or above (g < 0) the range: no preimage
    got = B.tgh_inverse(to_dev(t), (xi, omega, g, h)).cpu().numpy()
    ref = OG.tau_inverse((t - xi) / omega, g, h)
    np.testing.assert_array_equal(np.isnan(got), np.isnan(ref))
    ok = ~np.isnan(ref)
    # relative condition number of z = tau^-1(y): |y| / (|z| tau'(z)); it is
    # large near the edge of tau's range (h = 0, g y -> -1), where both sides
    # carry the rounding of y amplified by it
    y = (t[ok] - xi) / omega
    zr = ref[ok]
    cond = np.where(zr != 0.0, np.abs(y) / np.maximum(np.abs(zr) * OG.tau_prime(zr, g, h), 1e-300), 1.0)
    rel = np.abs(got[ok] - zr) / np.maximum(np.abs(zr), 1e-300)
    print(f"g={g} h={h}: max rel err {rel.max():.2e}, max cond {cond.max():.2e}, "
          f"{int((~ok).sum())} without preimage", flush=True)
    assert np.all(rel <= 1e-13 * np.maximum(cond, 10.0))


def test_inverse_empty_and_in_place():
    dev = device()
    empty = torch.empty(0, dtype=torch.float64, device=dev)
    B.tgh_inverse(empty, (0.0, 1.0, 0.2, 0.1))
    t = OG.sample_tgh(np.linspace(-3.0, 3.0, 301), 0.0, 1.0, 0.2, 0.1)
    dt = to_dev(t)
    B.tgh_inverse(dt, (0.0, 1.0, 0.2, 0.1), out=dt)
    np.testing.assert_allclose(dt.cpu().numpy(), np.linspace(-3.0, 3.0, 301), rtol=1e-12, atol=1e-14)


def tgh_problem(m, theta, tgh, kind="hilbert", extra=0):
    locs = synthetic.jittered_grid(m, synthetic.seed_for(8, synthetic.SEED_LOCS, extra))
    n = locs.shape[0]
    z = OL.sample_field(locs, theta, synthetic.standard_normal(n, synthetic.seed_for(8, synthetic.SEED_Z, extra)))
    t = OG.sample_tgh(z, *tgh)
    perm = OO.reorder(locs, kind)
    return locs[perm], t[perm]


@pytest.mark.parametrize("m,nb,tgh", [
    (40, 200, (0.5, 1.5, 0.4, 0.1)),
    (40, 200, (-1.0, 0.8, -0.6, 0.3)),
    (40, 320, (0.0, 1.0, 0.0, 0.0)),
    (90, 900, (0.2, 2.0, 0.3, 0.15)),
])
def test_loglik_tgh_against_oracle(m, nb, tgh):
    device()
    theta, tol = (1.0, 0.1, 0.5), 1e-9
    locs, t = tgh_problem(m, theta, tgh)
    n = locs.shape[0]
    plan = B.Plan(n, nb)
    ws = plan.workspace()
    z = torch.empty(n, dtype=torch.float64, device=ws.device)
    out = plan.loglik_tgh(ws, to_dev(locs), to_dev(t), theta, tgh, tol, z=z).cpu().numpy()
    zo = OG.tau_inverse((t - tgh[0]) / tgh[1], tgh[2], tgh[3])
    ref = OG.loglik_tgh(locs, t, theta, *tgh)
    jac = OG.log_jacobian(zo, tgh[1], tgh[2], tgh[3])
    err = abs(out[2] - ref)
    print(f"n={n} nb={nb} tgh={tgh}: gpu {out[2]!r} oracle {ref!r} |dl|={err:.2e} logjac {out[3]!r} / {jac!r}",
          flush=True)
    assert plan.status(ws)["code"] == 0
    assert abs(out[3] - jac) <= 1e-11 * max(1.0, abs(jac))
    np.testing.assert_allclose(z.cpu().numpy(), zo, rtol=1e-12, atol=1e-14)
    assert err <= n * max(1e-8, 0.1 * tol)
    if tgh[2] == 0.0 and tgh[3] == 0.0:  # Gaussian case: the plain likelihood of (t - xi)/omega, shifted
        g = plan.loglik(ws, to_dev(locs), to_dev((t - tgh[0]) / tgh[1]), theta, tol).cpu().numpy()
        assert abs(out[2] - (g[2] - n * np.log(tgh[1]))) <= 1e-12 * abs(g[2])


def test_loglik_tgh_without_preimage_is_minus_infinity():
    device()
    theta, tgh = (1.0, 0.1, 0.5), (0.0, 1.0, 1.0, 0.0)  # tau > -1
    locs, t = tgh_problem(20, theta, tgh)
    t[7] = -2.0
    assert OG.loglik_tgh(locs, t, theta, *tgh) == -np.inf
    plan = B.Plan(locs.shape[0], 100)
    ws = plan.workspace()
    out = plan.loglik_tgh(ws, to_dev(locs), to_dev(t), theta, tgh, 1e-9).cpu().numpy()
    assert out[2] == -np.inf


def test_loglik_tgh_mixed_precision():
    """The change of variables on a mixed plan: the Jacobian sum is the
    float64 plan's to the bit (it reads only z), and l_TGH lies within the
    mixed bound 1e-6 n of the oracle."""
    device()
    theta, tol, tgh = (1.0, 0.1, 0.5), 1e-9, (0.2, 2.0, 0.3, 0.15)
    locs, t = tgh_problem(60, theta, tgh, extra=1)
    n = locs.shape[0]
    ref = OG.loglik_tgh(locs, t, theta, *tgh)
    outs = {}
    for prec in ("fp64", "mixed_fp32"):
        plan = B.Plan(n, 360, precision=prec)
        ws = plan.workspace()
        outs[prec] = (plan.loglik_tgh(ws, to_dev(locs), to_dev(t), theta, tgh, tol).cpu().numpy(),
                      plan.status(ws)["code"])
    (o64, c64), (o32, c32) = outs["fp64"], outs["mixed_fp32"]
    print(f"tgh mixed n={n}: mixed {o32[2]!r} fp64 {o64[2]!r} oracle {ref!r} |dl|/n {abs(o32[2] - ref) / n:.2e}",
          flush=True)
    assert c64 == 0 and c32 == 0
    assert o32[3] == o64[3]
    assert abs(o32[2] - ref) <= 1e-6 * n
