"""Serving loop for l(theta) requests from many concurrent MLE fits.

Problems (ordered locations and observations) stay resident on the device.
A request names a problem and a theta; it is admitted when a workspace of its
plan's size can be taken from the pool without exceeding the HBM budget
(workspaces are reused across requests of the same plan shape), and runs on
one of the worker streams.  Requests that arrive while others run are
admitted as soon as a worker and memory free up, so evaluations of different
problems overlap on the device (continuous batching).  Every evaluation is
deterministic, so a result is bitwise the same alone and in the mix.

    python -m paper_2402_09356_amd.serve --bench     # the serving workload
"""
from __future__ import annotations

import argparse
import json
import math
import sys
import threading
import time
from concurrent.futures import Future
from dataclasses import dataclass, field

import numpy as np


@dataclass
class Problem:
    pid: int
    plan: object        # binding.Plan
    locs: object        # ordered locations, device tensor n x 2
    z: object           # ordered observations, device tensor n
    tol: float

    @property
    def key(self):
        return (self.plan.n, self.plan.nb, self.plan.maxrank)


@dataclass
class Request:
    pid: int
    theta: tuple
    submitted: float
    future: Future = field(default_factory=Future)
    started: float = 0.0
    finished: float = 0.0


class WorkspacePool:
    """Device workspaces by plan shape, under a byte budget.

    Idle workspaces are kept for reuse by requests of the same shape.  When a
    request needs a new workspace that the budget cannot hold, idle
    workspaces of other shapes are given up, least recently used first, until
    it fits (or none is left)."""

    def __init__(self, budget_bytes: int, device):
        self.budget = int(budget_bytes)
        self.device = device
        self.idle = []          # (key, workspace, bytes), least recently released first
        self.allocated = 0
        self.lock = threading.Lock()

    @property
    def free(self):
        out = {}
        for key, ws, _ in self.idle:
            out.setdefault(key, []).append(ws)
        return out

    def acquire(self, prob: Problem):
        import torch

        with self.lock:
            for i in range(len(self.idle) - 1, -1, -1):
                if self.idle[i][0] == prob.key:
                    return self.idle.pop(i)[1]
            need = int(prob.plan.ws_bytes)
            while self.allocated + need > self.budget and self.idle:
                _, ws, size = self.idle.pop(0)
                del ws
                self.allocated -= size
            if self.allocated + need > self.budget:
                return None
            self.allocated += need
        try:
            return torch.empty(need, dtype=torch.uint8, device=self.device)
        except RuntimeError:
            with self.lock:
                self.allocated -= need
            return None

    def release(self, prob: Problem, ws):
        with self.lock:
            self.idle.append((prob.key, ws, int(prob.plan.ws_bytes)))


class Server:
    def __init__(self, problems, workers: int = 8, hbm_budget_bytes: int = 200 << 30, device="cuda"):
        import torch

        self.problems = {p.pid: p for p in problems}
        self.pool = WorkspacePool(hbm_budget_bytes, torch.device(device))
        self.pending = []          # FIFO of requests not yet admitted
        self.cv = threading.Condition()
        self.stop = False
        self.completed = []
        self.workers = [threading.Thread(target=self._work, args=(w,), daemon=True) for w in range(workers)]
        self.device = device
        for t in self.workers:
            t.start()

    def submit(self, pid: int, theta) -> Request:
        req = Request(pid=pid, theta=tuple(float(t) for t in theta), submitted=time.perf_counter())
        with self.cv:
            self.pending.append(req)
            self.cv.notify()
        return req

    def _take(self):
        """First pending request (arrival order) whose workspace fits."""
        for i, req in enumerate(self.pending):
            ws = self.pool.acquire(self.problems[req.pid])
            if ws is not None:
                del self.pending[i]
                return req, ws
        return None, None

    def _work(self, w):
        import torch

        stream = torch.cuda.Stream(device=self.device)
        while True:
            with self.cv:
                while True:
                    if self.stop:
                        return
                    req, ws = self._take()
                    if req is not None:
                        break
                    self.cv.wait(timeout=0.05)
            prob = self.problems[req.pid]
            req.started = time.perf_counter()
            try:
                with torch.cuda.stream(stream):
                    out = torch.empty(3, dtype=torch.float64, device=self.device)
                    prob.plan.loglik(ws, prob.locs, prob.z, req.theta, prob.tol, out=out)
                    stream.synchronize()
                    val = float(out[2].item())
                req.finished = time.perf_counter()
                req.future.set_result(val)
            except Exception as exc:  # surfaced to the client
                req.finished = time.perf_counter()
                req.future.set_exception(exc)
            finally:
                self.pool.release(prob, ws)
                with self.cv:
                    self.completed.append(req)
                    self.cv.notify_all()

    def close(self):
        with self.cv:
            self.stop = True
            self.cv.notify_all()
        for t in self.workers:
            t.join()


def run_fits(server: Server, fits, think_mean_s: float, seed: int, max_evals: int, ftol: float = 1e-9):
    """Run Nelder-Mead fits as clients of the server, each in its own thread:
    each objective value is one request; between a result and the next
    request a fit waits an exponential think time (seeded per fit)."""
    from .mle import nelder_mead

    results = {}

    def client(idx, pid, start, nu):
        rng = np.random.default_rng(seed + idx)

        def objective(x):
            if think_mean_s > 0:
                time.sleep(rng.exponential(think_mean_s))
            th = (math.exp(x[0]), math.exp(x[1]), nu)
            return -server.submit(pid, th).future.result()

        res = nelder_mead(objective, np.log(start[:2]), step=0.1, ftol=ftol, max_evals=max_evals)
        results[idx] = res

    threads = [threading.Thread(target=client, args=(i, pid, start, nu)) for i, (pid, start, nu) in enumerate(fits)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    return results


def latency_stats(reqs):
    lat = np.array([r.finished - r.submitted for r in reqs]) * 1e3
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}


def _bench(args):
    import torch

    import synthetic
    from . import binding as B

    dev = torch.device("cuda:0")
    sizes = {10_000: (100, 400), 40_000: (200, 800), 90_000: (300, 900)}
    mix = [10_000] * args.n10 + [40_000] * args.n40 + [90_000] * args.n90
    problems, fits = [], []
    for pid, n in enumerate(mix):
        m, nb = sizes[n]
        locs = synthetic.jittered_grid(m, synthetic.seed_for(5, synthetic.SEED_LOCS, pid))
        z = synthetic.standard_normal(n, synthetic.seed_for(5, synthetic.SEED_Z, pid))
        dl = torch.from_numpy(locs).to(dev)
        perm = B.reorder(dl, "hilbert")
        ol, oz = B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))
        plan = B.Plan(n, nb, maxrank=args.maxrank)
        problems.append(Problem(pid, plan, ol, oz, args.tol))
        fits.append((pid, (0.5, 0.05, 0.5), 0.5))
    srv = Server(problems, workers=args.workers, hbm_budget_bytes=int(args.hbm_gib * 2**30))
    t0 = time.perf_counter()
    run_fits(srv, fits, args.think_ms * 1e-3, seed=5000, max_evals=args.evals_per_fit)
    wall = time.perf_counter() - t0
    srv.close()
    done = [r for r in srv.completed if r.future.exception() is None]
    out = {"metric": "served l(theta) evals/s", "value": len(done) / wall, "unit": "evals/s", "wall_s": wall,
           "latency": latency_stats(done), "workers": args.workers, "fits": len(fits),
           "mix": {"10k": args.n10, "40k": args.n40, "90k": args.n90}, "tol": args.tol, "precision": "fp64",
           "workspace_gib": srv.pool.allocated / 2**30}
    by_n = {}
    for r in done:
        by_n.setdefault(srv.problems[r.pid].plan.n, []).append(r)
    out["latency_by_n"] = {str(k): latency_stats(v) for k, v in sorted(by_n.items())}
    print(json.dumps(out))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench", action="store_true")
    ap.add_argument("--n10", type=int, default=19)
    ap.add_argument("--n40", type=int, default=10)
    ap.add_argument("--n90", type=int, default=3)
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--hbm-gib", type=float, default=200.0)
    ap.add_argument("--maxrank", type=int, default=256)
    ap.add_argument("--tol", type=float, default=1e-7)
    # each fit waits this long between a result and its next proposal; with 32
    # fits this offers about two thirds of the saturated capacity
    ap.add_argument("--think-ms", type=float, default=3500.0)
    ap.add_argument("--evals-per-fit", type=int, default=12)
    args = ap.parse_args()
    if args.bench:
        _bench(args)
    else:
        ap.print_help()
        sys.exit(2)


if __name__ == "__main__":
    main()
