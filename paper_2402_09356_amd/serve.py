"""Serving loop for l(theta) requests from many concurrent MLE fits.

Problems (ordered locations and observations) stay resident on the device.
A request names a problem and a theta; it is admitted when a workspace of its
plan's size can be taken from the pool without exceeding the HBM budget
(workspaces are reused across requests of the same plan shape), and runs on
one of the worker streams.  Requests that arrive while others run are
admitted as soon as a worker and memory free up, so evaluations of different
problems overlap on the device (continuous batching).  Every evaluation is
deterministic, so a result is bitwise the same alone and in the mix.

    python -m paper_2402_09356_amd.serve --bench     # the serving workload, FP64 and mixed
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


class _Stop(Exception):
    pass


def run_open_loop(server: Server, fits, rate: float | None, total: int, seed: int, max_evals: int = 100000,
                  progress=None):
    """Nelder-Mead fits as clients, gated by an open-loop arrival process.

    An arrival thread releases one ticket at each time of a Poisson process
    of the given rate (seeded); a fit that has its next proposal ready takes a
    ticket and submits that proposal as a request, so requests enter the
    server at the arrival times whatever the server's backlog (open loop),
    while each request still carries its fit's own next simplex point.  With
    rate None every fit submits as soon as its previous result is back
    (saturation, which measures capacity).  Stops once `total` requests have
    completed; returns the completed requests in completion order."""
    from .mle import nelder_mead

    import synthetic

    tickets = threading.Semaphore(0)
    stop = threading.Event()
    done = []
    lock = threading.Lock()

    def objective_for(pid, nu):
        def objective(x):
            if stop.is_set():
                raise _Stop()
            if rate is not None:
                while not tickets.acquire(timeout=0.05):
                    if stop.is_set():
                        raise _Stop()
            th = (math.exp(x[0]), math.exp(x[1]), nu)
            req = server.submit(pid, th)
            val = req.future.result()
            with lock:
                done.append(req)
                if progress is not None and len(done) % 100 == 0:
                    progress(len(done))
                if len(done) >= total:
                    stop.set()
            return -val
        return objective

    def client(pid, start, nu):
        while not stop.is_set():
            try:
                nelder_mead(objective_for(pid, nu), np.log(start[:2]), step=0.1, ftol=1e-9, max_evals=max_evals)
            except _Stop:
                return
            # a fit that converged starts again from its starting point

    def arrivals():
        gaps = synthetic.poisson_arrivals(4 * total + 100, rate, seed)
        t0 = time.perf_counter()
        for t in gaps:
            while not stop.is_set():
                dt = t - (time.perf_counter() - t0)
                if dt <= 0:
                    break
                time.sleep(min(dt, 0.05))
            if stop.is_set():
                return
            tickets.release()

    threads = [threading.Thread(target=client, args=f) for f in fits]
    if rate is not None:
        threads.append(threading.Thread(target=arrivals))
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    return done


def latency_stats(reqs):
    lat = np.array([r.finished - r.submitted for r in reqs]) * 1e3
    return {"count": int(lat.size), "p50_ms": float(np.percentile(lat, 50)), "p99_ms": float(np.percentile(lat, 99)),
            "mean_ms": float(lat.mean())}


def workload_problems(precision: str, tol: float, mix=(19, 10, 3), maxrank: int = 0, device="cuda:0"):
    """The serving workload: fits over three resident datasets (jittered grids,
    nu = 1/2, Hilbert order, Z ~ N(0, Sigma(1, 0.1, 1/2)) from the stored draws
    of the blocked dense oracle): n = 10,000 (nb = 400), 40,000 (nb = 800) and
    90,000 (nb = 900).  One resident problem per dataset; fit f of the mix
    starts from (0.5, 0.05) * exp(0.1 N(0, I)) (seeded), nu fixed at 1/2."""
    import os

    import torch

    import synthetic
    from . import binding as B

    root = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "tests", "golden")
    datasets = [("c5-10k", 5, 0, 400), ("c2-1", 2, 1, 800), ("c3", 3, 0, 900)]
    dev = torch.device(device)
    problems, fits = [], []
    for pid, (name, cfg, extra, nb) in enumerate(datasets):
        with open(os.path.join(root, f"large_{name}.json")) as fh:
            rec = json.load(fh)
        z = np.load(os.path.join(root, rec["z_file"]))
        locs = synthetic.jittered_grid(rec["m"], synthetic.seed_for(cfg, synthetic.SEED_LOCS, extra))
        dl = torch.from_numpy(locs).to(dev)
        perm = B.reorder(dl, "hilbert")
        ol, oz = B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))
        plan = B.Plan(rec["n"], nb, maxrank=maxrank, precision=precision)
        problems.append(Problem(pid, plan, ol, oz, tol))
    starts = synthetic.theta_perturbations((0.5, 0.05), sum(mix), synthetic.seed_for(5, synthetic.SEED_THETA), 0.1)
    f = 0
    for pid, count in enumerate(mix):
        for _ in range(count):
            fits.append((pid, tuple(float(v) for v in starts[f]), 0.5))
            f += 1
    return problems, fits


def _serve_once(precision, args):
    import torch

    problems, fits = workload_problems(precision, args.tol)
    out = {"precision": precision}
    log = lambda k: print(f"# {precision}: {k} completed", file=sys.stderr, flush=True)  # noqa: E731
    # capacity: every fit submits back to back
    srv = Server(problems, workers=args.workers, hbm_budget_bytes=int(args.hbm_gib * 2**30))
    run_open_loop(srv, fits, None, args.warmup, seed=1, progress=log)  # warm
    t0 = time.perf_counter()
    sat = run_open_loop(srv, fits, None, args.capacity_evals, seed=1, progress=log)
    cap = len(sat) / (time.perf_counter() - t0)
    srv.close()
    out["capacity_evals_per_s"] = cap
    rate = args.load * cap
    # open loop at `load` x capacity: warm-up, then the measured completions
    srv = Server(problems, workers=args.workers, hbm_budget_bytes=int(args.hbm_gib * 2**30))
    t_start = time.perf_counter()
    done = run_open_loop(srv, fits, rate, args.warmup + args.completions,
                         seed=synthetic_seed(args.seed), progress=log)
    srv.close()
    done.sort(key=lambda r: r.finished)
    measured = done[args.warmup:]
    # throughput over the measured window: from the last warm-up completion
    # to the last completion
    t_meas0 = done[args.warmup - 1].finished
    t_meas1 = measured[-1].finished
    ok = [r for r in measured if r.future.exception() is None and np.isfinite(r.future.result())]
    out.update({"arrival_rate_per_s": rate, "load": args.load, "completions": len(measured),
                "finite": len(ok), "evals_per_s": len(ok) / (t_meas1 - t_meas0),
                "wall_s": time.perf_counter() - t_start, "latency": latency_stats(measured),
                "workspace_gib": srv.pool.allocated / 2**30})
    by_n = {}
    for r in measured:
        by_n.setdefault(srv.problems[r.pid].plan.n, []).append(r)
    out["latency_by_n"] = {str(k): latency_stats(v) for k, v in sorted(by_n.items())}
    del problems
    torch.cuda.empty_cache()
    return out


def synthetic_seed(base: int) -> int:
    import synthetic

    return synthetic.seed_for(5, synthetic.SEED_ARRIVALS, base)


def _bench(args):
    res = {"metric": "served l(theta) evals/s", "unit": "evals/s", "workers": args.workers,
           "fits": {"10k": 19, "40k": 10, "90k": 3}, "tol": args.tol,
           "arrivals": f"open-loop Poisson at {args.load} x measured capacity, seeded"}
    for prec in ("fp64", "mixed_fp32"):
        res[prec] = _serve_once(prec, args)
        print(f"# {prec}: {json.dumps(res[prec])}", file=sys.stderr, flush=True)
    res["value"] = res["mixed_fp32"]["evals_per_s"]
    print(json.dumps(res))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--bench", action="store_true")
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--hbm-gib", type=float, default=200.0)
    ap.add_argument("--tol", type=float, default=1e-7)
    ap.add_argument("--load", type=float, default=0.8, help="arrival rate as a fraction of measured capacity")
    ap.add_argument("--capacity-evals", type=int, default=300)
    ap.add_argument("--warmup", type=int, default=100)
    ap.add_argument("--completions", type=int, default=1000)
    ap.add_argument("--seed", type=int, default=0)
    args = ap.parse_args()
    if args.bench:
        _bench(args)
    else:
        ap.print_help()
        sys.exit(2)


if __name__ == "__main__":
    main()
