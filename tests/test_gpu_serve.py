"""Serving: many concurrent requests over resident problems of different n;
admission by memory; every result bitwise equal to the same evaluation run
alone; open-loop arrivals driving Nelder-Mead clients; served results against
the dense oracle."""
import json
import os

import numpy as np
import pytest
import torch

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from paper_2402_09356_amd import binding as B
from paper_2402_09356_amd.serve import Problem, Server, latency_stats, run_fits, run_open_loop, workload_problems
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def _problems(precision="fp64"):
    out = []
    for pid, (m, nb) in enumerate([(40, 200), (50, 250), (60, 300)]):
        locs = synthetic.jittered_grid(m, synthetic.seed_for(5, synthetic.SEED_LOCS, pid))
        z = synthetic.standard_normal(m * m, synthetic.seed_for(5, synthetic.SEED_Z, pid))
        perm = OO.reorder(locs, "morton")
        out.append(Problem(pid, B.Plan(m * m, nb, precision=precision), to_dev(locs[perm]), to_dev(z[perm]), 1e-8))
    return out


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_results_alone_equal_results_in_the_mix(precision):
    device()
    probs = _problems(precision)
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


def test_open_loop_serving_against_the_oracle():
    """The serving workload's n = 10,000 and 40,000 problems (mixed
    precision), Nelder-Mead clients gated by a Poisson arrival stream; a few
    served 10k results checked against the dense oracle (|dl| <= 1e-6 n)."""
    device()
    problems, fits = workload_problems("mixed_fp32", 1e-7, mix=(4, 1, 0))
    srv = Server(problems[:2], workers=4)
    done = run_open_loop(srv, fits, rate=20.0, total=30, seed=synthetic.seed_for(5, synthetic.SEED_ARRIVALS))
    srv.close()
    assert len(done) >= 30
    assert all(np.isfinite(r.future.result()) for r in done)
    rec = json.load(open(os.path.join(GOLDEN, "large_c5-10k.json")))
    z = np.load(os.path.join(GOLDEN, rec["z_file"]))
    locs = synthetic.jittered_grid(100, synthetic.seed_for(5, synthetic.SEED_LOCS))
    ten = [r for r in done if r.pid == 0][:3]
    assert len(ten) == 3
    for r in ten:
        dense = OL.loglik_dense(locs, z, r.theta).loglik
        got = r.future.result()
        print(f"served 10k theta={r.theta}: {got!r} dense {dense!r} |dl|/n {abs(got - dense) / 1e4:.2e}", flush=True)
        assert abs(got - dense) <= 1e-6 * 10000
