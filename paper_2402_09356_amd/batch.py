"""Batched evaluation of many independent problems, and the tile-size tuner.

Each problem of a batch (its own n, locations, observations, theta and tile
size) is one l(theta) evaluation.  A batch goes to the library in one call
(`tlr_loglik_batched`), which runs the problems on worker streams, widest
first, so that the small kernels of different problems overlap on the device.
Results are bitwise those of one-at-a-time calls.

The tile size nb of a problem is picked by timing: for each candidate that
gives at least two tile rows, one warm evaluation is timed and the fastest
wins; the choice is cached per (n rounded to 1,000, tol, precision).

    python -m paper_2402_09356_amd.batch --bench    # 64 problems, n ~ U[2k, 20k]
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

NB_CANDIDATES = (160, 224, 320, 448, 640)
_nb_cache = {}


def autotune_nb(locs, z, theta, tol, candidates=NB_CANDIDATES, precision="fp64"):
    """Fastest tile size for this problem size (timed on the device)."""
    import torch

    from . import binding as B

    n = int(locs.shape[0])
    key = (round(n, -3), tol, precision)
    if key in _nb_cache:
        return _nb_cache[key]
    best, best_t = None, None
    for nb in candidates:
        if nb * 2 > n:
            continue
        plan = B.Plan(n, nb, maxrank=nb, precision=precision)
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


class Batch:
    """Problems of one batch, resident on the device, with their batch plan."""

    def __init__(self, locs, zs, thetas, nbs, tol, precision="fp64", maxrank=4096):
        from . import binding as B

        self.locs, self.zs, self.thetas, self.nbs, self.tol = list(locs), list(zs), list(thetas), list(nbs), tol
        self.precision = precision
        self.ns = [int(t.shape[0]) for t in self.locs]
        # maxrank above every nb: a tile never overflows its cap (nb x nb at most)
        self.plan = B.BatchPlan(self.ns, self.nbs, maxrank=maxrank, precision=precision)
        self.ws = None

    def loglik(self, workers=8):
        """count x 3 numpy array: {logdet, quad, l} per problem."""
        import torch

        if self.ws is None:
            self.ws = self.plan.workspace(self.locs[0].device)
        out = self.plan.loglik(self.ws, self.locs, self.zs, self.thetas, self.tol, workers=workers)
        torch.cuda.synchronize()
        return out.cpu().numpy()

    def sequential(self):
        """The same evaluations one at a time through tlr_loglik."""
        import torch

        from . import binding as B

        out = np.zeros((len(self.ns), 3))
        for p, (n, nb) in enumerate(zip(self.ns, self.nbs)):
            plan = B.Plan(n, nb, maxrank=4096, precision=self.precision)
            ws = plan.workspace(self.locs[p].device)
            out[p] = plan.loglik(ws, self.locs[p], self.zs[p], self.thetas[p], self.tol).cpu().numpy()
            del ws
        torch.cuda.synchronize()
        return out


def make_batch(count, seed, nmin=2000, nmax=20000, tol=1e-8, tune=True, device="cuda:0", precision="fp64"):
    """The batching workload: i.i.d. uniform locations, n ~ U{nmin..nmax},
    beta ~ U(0.03, 0.3), nu uniform over {1/2, 3/2, 5/2}, sigma2 = 1, Morton
    order; white-noise observations (the work of an evaluation does not depend
    on Z)."""
    import torch

    import synthetic
    from . import binding as B

    ns = synthetic.batch_sizes(count, nmin, nmax, synthetic.seed_for(seed, synthetic.SEED_LOCS))
    thetas = synthetic.batch_thetas(count, synthetic.seed_for(seed, synthetic.SEED_THETA))
    dev = torch.device(device)
    locs_l, z_l, th_l, nb_l = [], [], [], []
    for pid in range(count):
        n = int(ns[pid])
        locs = synthetic.uniform_points(n, synthetic.seed_for(seed, synthetic.SEED_LOCS, pid + 1))
        z = synthetic.standard_normal(n, synthetic.seed_for(seed, synthetic.SEED_Z, pid + 1))
        dl = torch.from_numpy(locs).to(dev)
        perm = B.reorder(dl, "morton")
        ol, oz = B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))
        th = tuple(float(v) for v in thetas[pid])
        nb = autotune_nb(ol, oz, th, tol, precision=precision) if tune else max(160, min(640, n // 16))
        locs_l.append(ol)
        z_l.append(oz)
        th_l.append(th)
        nb_l.append(nb)
    return Batch(locs_l, z_l, th_l, nb_l, tol, precision=precision)


def _bench(args):
    import torch

    rec = {"metric": "batched l(theta) evals/s", "unit": "evals/s", "problems": args.count, "workers": args.workers,
           "tol": args.tol}
    for prec in ("fp64", "mixed_fp32"):
        batch = make_batch(args.count, args.seed, tol=args.tol, precision=prec)
        torch.cuda.synchronize()
        batch.loglik(args.workers)  # warm
        t0 = time.perf_counter()
        bat = batch.loglik(args.workers)[:, 2]
        t_bat = time.perf_counter() - t0
        t0 = time.perf_counter()
        seq = batch.sequential()[:, 2]
        t_seq = time.perf_counter() - t0
        finite = int(np.sum(np.isfinite(bat)))
        codes = {}
        for p in range(len(bat)):
            if not np.isfinite(bat[p]):
                name = batch.plan.status(batch.ws, p)["name"]
                codes[name] = codes.get(name, 0) + 1
        same = bool(all((a == b) or (np.isnan(a) and np.isnan(b)) for a, b in zip(seq, bat)))
        # only finite results count as completed evaluations
        rec[prec] = {"evals_per_s": finite / t_bat, "finite_results": finite,
                     "nonfinite_results": len(bat) - finite, "nonfinite_status": codes,
                     "sequential_evals_per_s": int(np.sum(np.isfinite(seq))) / t_seq, "speedup": t_seq / t_bat,
                     "bitwise_equal_to_sequential": same, "nb": sorted(set(batch.nbs)),
                     "sum_n": int(sum(batch.ns))}
        del batch
        torch.cuda.empty_cache()
    rec["value"] = rec["mixed_fp32"]["evals_per_s"]
    print(json.dumps(rec))


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
