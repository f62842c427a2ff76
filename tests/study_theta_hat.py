"""Small-scale estimation study (paper Section 5.1.1, Fig. "plot1", and its
smooth variant in the appendix, Fig. "smooth"): for each correlation setting,
R seeded synthetic datasets of n = 1,600 jittered-grid locations; each dataset
is fitted by Nelder-Mead over (sigma2, beta, nu) with the GPU TLR likelihood
(nb = 320, tol = 1e-7, optimisation tolerance 1e-9) in every ordering (none,
Morton, Hilbert, KD-tree).  Reports per setting and ordering the quartiles of
sigma2-hat, beta-hat, nu-hat, f-hat = sigma2 beta^(-2 nu) and the number of
evaluations.

Runs on the GPU; the observations Z = L e come from the oracle's dense
Cholesky factor (this is why the driver sits with the tests).  Not collected
by pytest.

    python tests/study_theta_hat.py --reps 100 --out gpurun_out/study.jsonl
    python tests/study_theta_hat.py --summary gpurun_out/study.jsonl
"""
from __future__ import annotations

import argparse
import json
import math
import os
import queue
import sys
import threading
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

SETTINGS = {  # name: (nu, betas); sigma2 = 1 everywhere
    "rough": (0.5, (0.03, 0.1, 0.3)),
    "smooth": (1.0, (0.025, 0.075, 0.2)),
}
ORDERINGS = ("none", "morton", "hilbert", "kdtree")
M, NB, TOL, FTOL = 40, 320, 1e-7, 1e-9
START = (0.5, 0.05, 1.0)


def dataset(setting: str, ib: int, rep: int):
    import synthetic
    from oracle import likelihood as OL

    nu, betas = SETTINGS[setting]
    theta = (1.0, betas[ib], nu)
    extra = 1000 * (0 if setting == "rough" else 1) + 100 * ib + rep
    locs = synthetic.jittered_grid(M, synthetic.seed_for(10, synthetic.SEED_LOCS, extra))
    e = synthetic.standard_normal(M * M, synthetic.seed_for(10, synthetic.SEED_Z, extra))
    return theta, locs, OL.sample_field(locs, theta, e)


def run(args):
    import torch

    from oracle import ordering as OO
    from paper_2402_09356_amd import binding as B
    from paper_2402_09356_amd.mle import nelder_mead
    from paper_2402_09356_amd.serve import Problem, Server

    dev = torch.device("cuda:0")
    jobs, problems = [], []
    for setting in args.settings:
        for ib in range(3):
            for rep in range(args.reps):
                theta, locs, z = dataset(setting, ib, rep)
                for kind in ORDERINGS:
                    perm = np.arange(locs.shape[0]) if kind == "none" else OO.reorder(locs, kind)
                    pid = len(problems)
                    plan = B.Plan(M * M, NB, maxrank=NB // 2, dense_tiles=True)
                    problems.append(Problem(pid, plan, torch.from_numpy(locs[perm].copy()).to(dev),
                                            torch.from_numpy(z[perm].copy()).to(dev), TOL))
                    jobs.append((pid, setting, theta, rep, kind))
    print(f"# {len(jobs)} fits", flush=True)
    server = Server(problems, workers=args.workers, hbm_budget_bytes=64 << 30, device="cuda:0")
    todo = queue.Queue()
    for j in jobs:
        todo.put(j)
    out = open(args.out, "w")
    lock = threading.Lock()
    done = [0]
    t0 = time.perf_counter()

    def client():
        while True:
            try:
                pid, setting, theta, rep, kind = todo.get_nowait()
            except queue.Empty:
                return

            def objective(x):
                th = tuple(math.exp(v) for v in x)
                val = server.submit(pid, th).future.result()
                return -val if math.isfinite(val) else math.inf

            res = nelder_mead(objective, np.log(START), step=0.1, ftol=args.ftol, max_evals=args.max_evals)
            th = tuple(math.exp(v) for v in res.x)
            rec = {"setting": setting, "theta_true": list(theta), "rep": rep, "ordering": kind,
                   "theta_hat": list(th), "f_hat": th[0] * th[1] ** (-2.0 * th[2]), "loglik": -res.f,
                   "evals": res.evals, "converged": res.converged}
            with lock:
                out.write(json.dumps(rec) + "\n")
                done[0] += 1
                if done[0] % 50 == 0:
                    out.flush()
                    print(f"# {done[0]}/{len(jobs)} fits, {time.perf_counter() - t0:.0f} s", flush=True)

    threads = [threading.Thread(target=client) for _ in range(args.clients)]
    for t in threads:
        t.start()
    for t in threads:
        t.join()
    server.close()
    out.close()
    evals = len(server.completed)
    print(f"# done: {len(jobs)} fits, {evals} evaluations in {time.perf_counter() - t0:.1f} s", flush=True)


def summary(path):
    recs = [json.loads(line) for line in open(path)]
    cells = {}
    for r in recs:
        cells.setdefault((r["setting"], r["theta_true"][1], r["ordering"]), []).append(r)
    print("| setting | beta | ordering | fits | sigma2-hat | beta-hat | nu-hat | f-hat / f | evals |")
    print("|---|---|---|---|---|---|---|---|---|")

    def q(v):
        a = np.percentile(v, [25, 50, 75])
        return f"{a[1]:.3g} [{a[0]:.3g}, {a[2]:.3g}]"

    for key in sorted(cells, key=lambda k: (k[0], k[1], ORDERINGS.index(k[2]))):
        rs = cells[key]
        th = np.array([r["theta_hat"] for r in rs])
        tt = rs[0]["theta_true"]
        f = tt[0] * tt[1] ** (-2.0 * tt[2])
        print(f"| {key[0]} | {key[1]} | {key[2]} | {len(rs)} | {q(th[:, 0])} | {q(th[:, 1])} | {q(th[:, 2])} | "
              f"{q(np.array([r['f_hat'] for r in rs]) / f)} | {q(np.array([r['evals'] for r in rs]))} |")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--reps", type=int, default=100)
    ap.add_argument("--settings", nargs="+", default=["rough", "smooth"], choices=sorted(SETTINGS))
    ap.add_argument("--workers", type=int, default=8)
    ap.add_argument("--clients", type=int, default=64)
    ap.add_argument("--max-evals", type=int, default=1000)
    ap.add_argument("--ftol", type=float, default=FTOL)
    ap.add_argument("--out", default="gpurun_out/study.jsonl")
    ap.add_argument("--summary")
    args = ap.parse_args()
    if args.summary:
        summary(args.summary)
    else:
        run(args)


if __name__ == "__main__":
    main()
