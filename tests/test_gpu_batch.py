"""Batching: many independent problems (own n, theta, nu, tile size) evaluated
concurrently; results bitwise those of sequential calls and within the
tolerance bound of the dense oracle."""
import numpy as np
import pytest

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from oracle import tlr as OT
from paper_2402_09356_amd import binding as B
from paper_2402_09356_amd.batch import batch_loglik, sequential_loglik
from paper_2402_09356_amd.serve import Problem
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


def test_batch_equals_sequential_and_oracle():
    device()
    tol = 1e-8
    problems, thetas, host = [], [], []
    for pid, (n, nb, th) in enumerate(CASES):
        locs = synthetic.uniform_points(n, 4000 + 10 * pid + 1)
        e = synthetic.standard_normal(n, 4000 + 10 * pid + 2)
        z = OL.sample_field(locs, th, e)
        perm = OO.reorder(locs, "morton")
        problems.append(Problem(pid, B.Plan(n, nb, maxrank=nb), to_dev(locs[perm]), to_dev(z[perm]), tol))
        thetas.append(th)
        host.append((locs[perm], z[perm]))
    seq = sequential_loglik(problems, thetas)
    bat = batch_loglik(problems, thetas, workers=4)
    for pid, (a, b) in enumerate(zip(seq, bat)):
        assert a == b, (pid, a, b)
    # every case is SPD on the oracle's side, dense and tile-truncated: a
    # non-finite GPU result is a failure
    for (locs, z), th, got, (n, nb, _) in zip(host, thetas, bat, CASES):
        dense = OL.loglik_dense(locs, z, th).loglik
        comp, _ = OT.compressed_loglik(locs, z, th, nb, tol, maxrank=nb)
        assert np.isfinite(got), (n, th, got, dense)
        assert abs(got - dense) <= bound(n, tol, comp.loglik - dense), (n, th, got, dense)
