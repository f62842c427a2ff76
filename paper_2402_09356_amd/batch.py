"""Batched evaluation of many independent problems, and the tile-size tuner.

Each problem of a batch (its own n, locations, observations, theta and tile
size) is one l(theta) evaluation; the evaluations run concurrently on the
serving loop's worker streams, so the small kernels of different problems
overlap on the device.  Results are bitwise those of one-at-a-time calls.

The tile size nb of a problem is picked by timing: for each candidate that
gives at least two tile rows, one warm evaluation is timed and the fastest
wins; the choice is cached per (n rounded to 1,000, tol).

    python -m paper_2402_09356_amd.batch --bench    # 64 problems, n ~ U[2k, 20k]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

NB_CANDIDATES = (160, 224, 320, 448, 640)
_nb_cache = {}


def autotune_nb(locs, z, theta, tol, candidates=NB_CANDIDATES, maxrank=0):
    """Fastest tile size for this problem size (timed on the device)."""
    import torch

    from . import binding as B

    n = int(locs.shape[0])
    key = (round(n, -3), tol)
    if key in _nb_cache:
        return _nb_cache[key]
    best, best_t = None, None
    for nb in candidates:
        if nb * 2 > n:
            continue
        plan = B.Plan(n, nb, maxrank=maxrank, dense_tiles=True)
        ws = plan.workspace(locs.device)
        out = torch.empty(3, dtype=torch.float64, device=locs.device)
        plan.loglik(ws, locs, z, theta, tol, out=out)  # warm
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.loglik(ws, locs, z, theta, tol, out=out)
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0
        del ws
        if best_t is None or dt < best_t:
            best, best_t = nb, dt
    if best is None:
        best = max(16, n // 2)
    _nb_cache[key] = best
    return best


def batch_loglik(problems, thetas, workers=8, hbm_budget_bytes=200 << 30):
    """l(theta_p) for every problem p, evaluated concurrently.

    problems: serve.Problem list; thetas: one theta per problem."""
    from .serve import Server

    srv = Server(problems, workers=workers, hbm_budget_bytes=hbm_budget_bytes)
    try:
        reqs = [srv.submit(p.pid, th) for p, th in zip(problems, thetas)]
        return [r.future.result() for r in reqs]
    finally:
        srv.close()


def sequential_loglik(problems, thetas):
    import torch

    out = []
    for p, th in zip(problems, thetas):
        ws = p.plan.workspace(p.z.device)
        out.append(float(p.plan.loglik(ws, p.locs, p.z, th, p.tol)[2].item()))
        del ws
    torch.cuda.synchronize()
    return out


def make_batch(count, seed, nmin=2000, nmax=20000, tol=1e-8, tune=True, device="cuda:0"):
    """The batching workload: i.i.d. uniform locations, n ~ U{nmin..nmax},
    beta ~ U(0.03, 0.3), nu uniform over {1/2, 3/2, 5/2}, sigma2 = 1, Morton."""
    import torch

    import synthetic
    from . import binding as B
    from .serve import Problem

    rng = np.random.default_rng(seed)
    ns = rng.integers(nmin, nmax + 1, size=count)
    betas = rng.uniform(0.03, 0.3, size=count)
    nus = rng.choice([0.5, 1.5, 2.5], size=count)
    problems, thetas = [], []
    dev = torch.device(device)
    for pid in range(count):
        n = int(ns[pid])
        locs = synthetic.uniform_points(n, seed * 1000 + 10 * pid + 1)
        z = synthetic.standard_normal(n, seed * 1000 + 10 * pid + 2)
        dl = torch.from_numpy(locs).to(dev)
        perm = B.reorder(dl, "morton")
        ol, oz = B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))
        th = (1.0, float(betas[pid]), float(nus[pid]))
        nb = autotune_nb(ol, oz, th, tol) if tune else max(160, min(640, n // 16))
        # over-rank tiles are kept dense (uniform points at tol = 1e-8 can
        # exceed nb/2), so no evaluation stops at the rank cap
        problems.append(Problem(pid, B.Plan(n, nb, dense_tiles=True), ol, oz, tol))
        thetas.append(th)
    return problems, thetas


def _bench(args):
    import torch

    problems, thetas = make_batch(args.count, args.seed, tol=args.tol)
    torch.cuda.synchronize()
    batch_loglik(problems[:4], thetas[:4], workers=args.workers)  # warm
    t0 = time.perf_counter()
    seq = sequential_loglik(problems, thetas)
    t_seq = time.perf_counter() - t0
    t0 = time.perf_counter()
    bat = batch_loglik(problems, thetas, workers=args.workers)
    t_bat = time.perf_counter() - t0
    same = all((a == b) or (np.isnan(a) and np.isnan(b)) for a, b in zip(seq, bat))
    finite = int(sum(np.isfinite(v) for v in bat))
    # only finite results count as completed evaluations
    print(json.dumps({"metric": "batched l(theta) evals/s", "value": finite / t_bat, "unit": "evals/s",
                      "finite_results": finite, "nonfinite_results": len(bat) - finite,
                      "sequential_evals_per_s": int(sum(np.isfinite(v) for v in seq)) / t_seq,
                      "speedup": t_seq / t_bat,
                      "problems": len(problems), "workers": args.workers, "bitwise_equal": same,
                      "nb": sorted({p.plan.nb for p in problems}), "tol": args.tol, "precision": "fp64",
                      "sum_n": int(sum(p.plan.n for p in problems))}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench", action="store_true")
    ap.add_argument("--count", type=int, default=64)
    ap.add_argument("--seed", type=int, default=4)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--tol", type=float, default=1e-8)
    args = ap.parse_args()
    if not args.bench:
        ap.print_help()
        raise SystemExit(2)
    _bench(args)


if __name__ == "__main__":
    main()
