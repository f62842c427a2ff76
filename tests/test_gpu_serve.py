"""Serving: many concurrent requests over resident problems of different n;
admission by memory; every result bitwise equal to the same evaluation run
alone."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import ordering as OO
from paper_2402_09356_amd import binding as B
from paper_2402_09356_amd.serve import Problem, Server, latency_stats, run_fits
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


def _problems():
    out = []
    for pid, (m, nb) in enumerate([(40, 200), (50, 250), (60, 300)]):
        locs = synthetic.jittered_grid(m, synthetic.seed_for(5, synthetic.SEED_LOCS, pid))
        z = synthetic.standard_normal(m * m, synthetic.seed_for(5, synthetic.SEED_Z, pid))
        perm = OO.reorder(locs, "morton")
        out.append(Problem(pid, B.Plan(m * m, nb), to_dev(locs[perm]), to_dev(z[perm]), 1e-8))
    return out


def test_results_alone_equal_results_in_the_mix():
    device()
    probs = _problems()
    thetas = synthetic.theta_perturbations((1.0, 0.1, 0.5), 24, 77)
    jobs = [(i % 3, tuple(float(t) for t in thetas[i])) for i in range(24)]
    alone = []
    for pid, th in jobs:
        p = probs[pid]
        ws = p.plan.workspace()
        alone.append(p.plan.loglik(ws, p.locs, p.z, th, p.tol).cpu().numpy()[2])
        del ws
    torch.cuda.synchronize()
    # budget for about two workspaces at once: admission must hold requests back
    budget = int(1.2 * max(p.plan.ws_bytes for p in probs) + max(p.plan.ws_bytes for p in probs))
    srv = Server(probs, workers=4, hbm_budget_bytes=budget)
    reqs = [srv.submit(pid, th) for pid, th in jobs]
    mixed = [r.future.result(timeout=120) for r in reqs]
    srv.close()
    assert srv.pool.allocated <= budget
    for a, b in zip(alone, mixed):
        assert np.isfinite(a) and a == b, (a, b)
    st = latency_stats(reqs)
    assert st["count"] == 24 and st["p99_ms"] >= st["p50_ms"] > 0


def test_fits_as_clients():
    device()
    probs = _problems()
    srv = Server(probs, workers=3)
    res = run_fits(srv, [(0, (0.5, 0.05), 0.5), (1, (0.5, 0.05), 0.5), (2, (0.5, 0.05), 0.5)], think_mean_s=0.001,
                   seed=1, max_evals=15)
    srv.close()
    assert len(res) == 3 and all(np.isfinite(r.f) for r in res.values())
    assert len(srv.completed) == sum(r.evals for r in res.values())
