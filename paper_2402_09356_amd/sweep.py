"""Rank and storage sweep over orderings (the medium-scale configuration).

For each cell (nu, beta, ordering, nb, tol) on an m x m jittered grid: the
per-tile ranks after compression, their histogram, the off-diagonal storage
in MB (2 nb r 8 bytes per low-rank tile, nb^2 8 per dense one: the quantity of the
paper's Table "memory"), l(theta_true) and the time of one evaluation.  Ranks do not depend
on the observations, so Z is white noise here.

    python -m paper_2402_09356_amd.sweep --m 200 --nu 0.5 --beta 0.03 0.1 0.3 \\
        --orderings random morton hilbert kdtree --nb 800 --tol 1e-7
"""
from __future__ import annotations

import argparse
import json
import time

import numpy as np

BINS = (0, 1, 11, 26, 51, 101, 201, 10**9)


def run_cell(m, nu, beta, kind, nb, tol, exact_ranks=False, seed_cfg=2, cell=0, dense_tiles=False):
    import torch

    import synthetic
    from . import binding as B

    dev = torch.device("cuda:0")
    n = m * m
    locs = synthetic.jittered_grid(m, synthetic.seed_for(seed_cfg, synthetic.SEED_LOCS, cell))
    z = synthetic.standard_normal(n, synthetic.seed_for(seed_cfg, synthetic.SEED_Z, cell))
    dl = torch.from_numpy(locs).to(dev)
    perm = B.reorder(dl, kind, synthetic.seed_for(seed_cfg, synthetic.SEED_ORDER, cell))
    ol, oz = B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))
    plan = B.Plan(n, nb, maxrank=nb // 2, dense_tiles=dense_tiles, truncation="svd" if exact_ranks else "qrcp")
    ws = plan.workspace(dev)
    theta = (1.0, beta, nu)
    out = plan.loglik(ws, ol, oz, theta, tol)  # warm
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    out = plan.loglik(ws, ol, oz, theta, tol)
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    st = plan.status(ws)
    nt = plan.nt
    # ranks, l and the time all come from the same (timed) evaluation
    r = plan.ranks(ws)
    rk = np.asarray([int(r[i, j]) for i in range(nt) for j in range(i)])
    over = int(np.sum(rk == -1))
    dense = int(np.sum(rk == -2))
    low = rk[rk >= 0]
    hist = np.histogram(low, bins=np.asarray(BINS))[0].tolist()
    storage_mb = float(2 * nb * low.sum() * 8 / 1e6 + (over + dense) * nb * nb * 8 / 1e6)
    return {"n": n, "nu": nu, "beta": beta, "ordering": kind, "nb": nb, "tol": tol,
            "loglik": float(out[2].item()), "eval_s": dt, "status": st["code"],
            "rank_mean": float(low.mean()) if low.size else None, "rank_max": int(low.max()) if low.size else None,
            "hist_bins": list(BINS), "hist": hist, "overflow_tiles": over, "dense_tiles": dense,
            "offdiag_storage_MB": storage_mb,
            "rank_mode": "singular values" if exact_ranks else "pivoted QR"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--m", type=int, default=200)
    ap.add_argument("--nu", type=float, nargs="+", default=[0.5])
    ap.add_argument("--beta", type=float, nargs="+", default=[0.03, 0.1, 0.3])
    ap.add_argument("--orderings", nargs="+", default=["random", "morton", "hilbert", "kdtree"])
    ap.add_argument("--nb", type=int, nargs="+", default=[800])
    ap.add_argument("--tol", type=float, nargs="+", default=[1e-7])
    ap.add_argument("--exact-ranks", action="store_true")
    ap.add_argument("--dense-tiles", action="store_true", help="keep over-rank tiles dense")
    args = ap.parse_args()
    cell = 0
    for nu in args.nu:
        for beta in args.beta:
            cell += 1
            for kind in args.orderings:
                for nb in args.nb:
                    for tol in args.tol:
                        rec = run_cell(args.m, nu, beta, kind, nb, tol, args.exact_ranks, cell=cell,
                                       dense_tiles=args.dense_tiles)
                        print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
