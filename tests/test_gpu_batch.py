"""Batching: many independent problems (own n, theta, nu, tile size) in one
tlr_loglik_batched call; results bitwise those of one-at-a-time tlr_loglik
calls and, for every problem, within the tolerance bound of the dense
oracle (float64), or within 1e-6 n (float32 factors, nu = 1/2 problems)."""
import numpy as np
import pytest

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from oracle import tlr as OT
from paper_2402_09356_amd.batch import Batch
from tests.gpu_util import device, to_dev
from tests.test_gpu_loglik import bound

pytestmark = pytest.mark.gpu

CASES = [  # n, nb, theta
    (900, 160, (1.0, 0.05, 0.5)),
    (1337, 224, (1.0, 0.03, 1.5)),
    (2000, 320, (1.0, 0.1, 0.5)),
    (1500, 160, (1.0, 0.02, 2.5)),
    (2400, 448, (1.0, 0.06, 1.5)),
    (1100, 224, (2.0, 0.08, 0.5)),
]


def _problems():
    host, locs_d, z_d = [], [], []
    for pid, (n, nb, th) in enumerate(CASES):
        locs = synthetic.uniform_points(n, 4000 + 10 * pid + 1)
        e = synthetic.standard_normal(n, 4000 + 10 * pid + 2)
        z = OL.sample_field(locs, th, e)
        perm = OO.reorder(locs, "morton")
        host.append((locs[perm], z[perm]))
        locs_d.append(to_dev(locs[perm]))
        z_d.append(to_dev(z[perm]))
    return host, locs_d, z_d


def test_batch_equals_sequential_and_oracle():
    device()
    tol = 1e-8
    host, locs_d, z_d = _problems()
    batch = Batch(locs_d, z_d, [c[2] for c in CASES], [c[1] for c in CASES], tol)
    bat = batch.loglik(workers=4)
    seq = batch.sequential()
    assert bat.tobytes() == seq.tobytes()
    # every case is SPD on the oracle's side, dense and tile-truncated: a
    # non-finite GPU result is a failure
    for (locs, z), got, (n, nb, th) in zip(host, bat[:, 2], CASES):
        dense = OL.loglik_dense(locs, z, th).loglik
        comp, _ = OT.compressed_loglik(locs, z, th, nb, tol, maxrank=nb)
        print(f"batch n={n} nu={th[2]}: gpu {got!r} dense {dense!r}", flush=True)
        assert np.isfinite(got), (n, th, got, dense)
        assert abs(got - dense) <= bound(n, tol, comp.loglik - dense), (n, th, got, dense)


def test_mixed_batch():
    device()
    tol = 1e-8
    host, locs_d, z_d = _problems()
    batch = Batch(locs_d, z_d, [c[2] for c in CASES], [c[1] for c in CASES], tol, precision="mixed_fp32")
    bat = batch.loglik(workers=3)
    seq = batch.sequential()
    assert bat.tobytes() == seq.tobytes()
    for (locs, z), got, (n, nb, th) in zip(host, bat[:, 2], CASES):
        dense = OL.loglik_dense(locs, z, th).loglik
        print(f"mixed batch n={n} nu={th[2]}: gpu {got!r} dense {dense!r} |dl|/n {abs(got - dense) / n:.2e}",
              flush=True)
        assert np.isfinite(got)
        if th[2] == 0.5:
            assert abs(got - dense) <= 1e-6 * n
