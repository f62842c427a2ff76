"""Throughput of l(theta) evaluations through the TLR path on one MI355X.

Workload (default): n = 90,000 locations on a 300 x 300 jittered grid in the
unit square, Matern nu = 1/2, beta = 0.1, sigma2 = 1, Hilbert ordering, tiles
of nb = 900 (100 x 100 tiles), accuracy threshold tol = 1e-7.  One step is one
full evaluation: covariance generation, per-tile compression, TLR Cholesky,
forward solve, log-determinant and l, at parameters theta_true * exp(0.2 N(0,I))
(seeded; a fresh theta every step, as an optimiser would propose).  Inputs
(ordered locations, observations) are resident in HBM before timing starts.

`value` is evaluations per second with one evaluation at a time (the timed
steps, where the launch timer measures each kernel on its stream).
Evaluations are independent (each its own theta), and one evaluation leaves
most compute units idle during the factorisation, so the same steps are then
run again with three in flight, each on its own stream and workspace; that
throughput, its per-evaluation latency and a bitwise check against the
one-at-a-time results are reported under "concurrent".

Prints one JSON line.  --config c1 runs the small 1,600-point case instead.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

CONFIGS = {
    # name: (grid m, nb, tol, theta_true, ordering, config number for seeds)
    "c1": (40, 200, 1e-9, (1.0, 0.1, 0.5), "morton", 1),
    "c3": (300, 900, 1e-7, (1.0, 0.1, 0.5), "hilbert", 3),
}


def cpu_baseline(locs_ordered: np.ndarray, z_ordered: np.ndarray, theta, n_full: int, sample_n: int):
    """Dense oracle l on the first sample_n ordered points, scaled to n_full by n^3."""
    import oracle.likelihood as OL

    sub_l, sub_z = locs_ordered[:sample_n], z_ordered[:sample_n]
    t0 = time.perf_counter()
    OL.loglik_dense(sub_l, sub_z, theta)
    dt = time.perf_counter() - t0
    scale = (n_full / sample_n) ** 3
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    threads = int(os.environ.get("OMP_NUM_THREADS", cores))
    return {"value": 1.0 / (dt * scale), "unit": "evals/s", "cores": min(cores, threads), "kind": "oracle",
            "sample": f"dense float64 oracle l (Matern matrix, LAPACK Cholesky, solve) on the first {sample_n} "
                      f"ordered points: {dt:.2f} s; evals/s scaled to n={n_full} by (n/{sample_n})^3"}


# MI355X published peaks used for roofline fractions
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6      # FP64 matrix (MFMA) and FP64 vector alike
VALU_KERNELS = ("k_chol_small", "k_trsm_rows", "k_trsv_tile", "k_qrcp_trunc", "k_qrcp_reg", "k_jacobi_svd",
                "k_lr_gemv", "k_gen_tiles")


def measured_traffic(kernel: str, workload: str):
    """HBM bytes per launch of `kernel` from the committed counter summary
    (FETCH_SIZE + WRITE_SIZE scaled by the copy-kernel factor), if it was
    taken for these kernel sources and this workload; else None."""
    path = os.path.join(ROOT, "profiles", "traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    from paper_2402_09356_amd.traffic import source_digest

    if rec.get("source_sha256") != source_digest() or rec.get("workload") != workload:
        return None
    ks = rec.get("kernels", {})
    if kernel in ks:
        return float(ks[kernel]["hbm_bytes_per_launch"])
    # a launch-timer class such as k_gemm_lds<N,N> covers the instantiations
    # k_gemm_lds<N,N,BM,BN> the counters list apart: their dispatch-weighted mean
    pre = kernel[:-1] + "," if kernel.endswith(">") else None
    parts = [v for name, v in ks.items() if pre and name.startswith(pre)]
    n = sum(v["dispatches"] for v in parts)
    return None if n == 0 else sum(v["hbm_bytes_per_launch"] * v["dispatches"] for v in parts) / n


def roofline(stats, workload: str, warm_stats=None):
    """Roofline record of the kernel with the largest total launch time (the
    one class timed in the timed steps); its share of all kernel time comes
    from the warm-up steps, where every class is timed."""
    top = stats[0]
    share_src = warm_stats if warm_stats else stats
    share = next((s["total_ms"] for s in share_src if s["name"] == top["name"]), 0.0) / max(
        sum(s["total_ms"] for s in share_src), 1e-30)
    if top["exact_launches"] == 0 or top["exact_ms"] <= 0.0:
        return {"kernel": top["name"], "bound": None, "achieved": None, "peak": None, "unit": None, "frac": None,
                "traffic": None, "avg_launch_us": 1e3 * top["total_ms"] / max(top["launches"], 1),
                "launches": top["launches"], "note": "work of this kernel is decided on the device"}
    sec = top["exact_ms"] * 1e-3
    note = None
    t_flops = top["flops"] / (PEAK_FP64_TFLOPS * 1e12)
    t_bytes = top["bytes"] / (PEAK_HBM_GBS * 1e9)
    per = top["exact_launches"]
    if t_bytes >= t_flops:
        bound, achieved, peak, unit = "hbm", top["bytes"] / sec / 1e9, PEAK_HBM_GBS, "GB/s"
    else:
        bound = "alu" if top["name"] in VALU_KERNELS else "mfma"
        achieved, peak, unit = top["flops"] / sec / 1e12, PEAK_FP64_TFLOPS, "TFLOP/s"
    if achieved / peak < 0.05 and top["flops"] / sec / 1e12 / PEAK_FP64_TFLOPS < 0.05:
        note = ("latency-bound: neither HBM nor FP64 throughput limits it; its time is the dependent chain "
                "of the largest problem in each batched launch")
    return {"kernel": top["name"], "bound": bound, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": achieved / peak, "traffic": measured_traffic(top["name"], workload), "note": note,
            "avg_launch_us": 1e3 * top["total_ms"] / max(top["launches"], 1), "launches": top["launches"],
            "exact_launches": per, "exact_avg_launch_us": 1e3 * top["exact_ms"] / per,
            "algorithmic_bytes_per_launch": top["bytes"] / per, "algorithmic_flops_per_launch": top["flops"] / per,
            "share_of_kernel_time": share}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--config", default="c3", choices=sorted(CONFIGS))
    ap.add_argument("--precision", default="fp64", choices=["fp64"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--concurrency", type=int, default=3,
                    help="after the timed steps, run them again with this many evaluations in flight "
                         "(each on its own stream and workspace) and report that throughput beside")
    ap.add_argument("--copy-probe-mib", type=int, default=0,
                    help="run one plain device copy of this size before warmup (counter calibration)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU; multi-GPU runs are not part of this build", file=sys.stderr)
        sys.exit(2)

    import torch

    import synthetic
    from paper_2402_09356_amd import binding as B

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    m, nb, tol, theta_true, kind, cfg = CONFIGS[args.config]
    n = m * m
    locs = synthetic.jittered_grid(m, synthetic.seed_for(cfg, synthetic.SEED_LOCS))
    # white-noise observations: the work of an evaluation does not depend on Z
    z = synthetic.standard_normal(n, synthetic.seed_for(cfg, synthetic.SEED_Z))
    thetas = synthetic.theta_perturbations(theta_true, args.warmup + args.steps,
                                           synthetic.seed_for(cfg, synthetic.SEED_THETA))

    dlocs = torch.from_numpy(locs).to(dev)
    perm = B.reorder(dlocs, kind, synthetic.seed_for(cfg, synthetic.SEED_ORDER))
    olocs, oz = B.apply_perm(perm, dlocs, torch.from_numpy(z).to(dev))
    plan = B.Plan(n, nb, precision=args.precision)
    ws = plan.workspace(dev)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    conc = max(1, args.concurrency)
    extra_ws = [plan.workspace(dev) for _ in range(conc - 1)]
    torch.cuda.synchronize()
    print(f"# workspace {plan.ws_bytes / 2**30:.2f} GiB, nt={plan.nt}, maxrank={plan.maxrank}", file=sys.stderr,
          flush=True)
    if args.copy_probe_mib > 0:
        src = torch.ones(args.copy_probe_mib << 17, dtype=torch.float64, device=dev)
        dst = torch.empty_like(src)
        dst.copy_(src)
        torch.cuda.synchronize()
        del src, dst
    # warm-up steps time every kernel class; the timed steps then time only
    # the class that dominated, so the timer's events sit on that kernel's
    # launches alone and the others run as they do untimed
    B.kstats_select(None)
    B.kstats_enable(True)
    B.kstats_reset()
    for w in range(args.warmup):
        plan.loglik(ws, olocs, oz, thetas[w], tol, out=out)
        torch.cuda.synchronize()
        print(f"# warmup {w}: l={out[2].item():.6f}", file=sys.stderr, flush=True)
    warm_stats = B.kstats()
    B.kstats_enable(False)
    timed_class = warm_stats[0]["name"] if warm_stats and warm_stats[0]["launches"] > 0 else None
    for k in warm_stats[:16]:
        print(f"# warm-up {k['name']:20s} launches {k['launches']:7d}  total {k['total_ms']:10.2f} ms  "
              f"avg {1e3 * k['total_ms'] / max(k['launches'], 1):9.2f} us", file=sys.stderr)
    lat = [0.0] * args.steps
    lls = [0.0] * args.steps
    B.kstats_select(timed_class)
    B.kstats_enable(True)
    B.kstats_reset()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for k in range(args.steps):
        t0 = time.perf_counter()
        plan.loglik(ws, olocs, oz, thetas[args.warmup + k], tol, out=out)
        torch.cuda.synchronize()
        lat[k] = time.perf_counter() - t0
        lls[k] = out[2].item()
        print(f"# step {k}: {lat[k] * 1e3:.1f} ms l={lls[k]:.6f}", file=sys.stderr, flush=True)
    torch.cuda.synchronize()
    total = time.perf_counter() - t_start
    stats = B.kstats()
    B.kstats_enable(False)
    B.kstats_select(None)
    concurrent = None
    if conc > 1:
        # the same steps again with `conc` evaluations in flight, one stream and
        # one workspace each; results must equal the one-at-a-time ones
        import threading

        wss = [ws] + extra_ws
        clat = [0.0] * args.steps
        cll = [0.0] * args.steps

        def worker(w):
            stream = torch.cuda.Stream(device=dev)
            with torch.cuda.stream(stream):
                o = torch.empty(3, dtype=torch.float64, device=dev)
                for k in range(w, args.steps, conc):
                    t0 = time.perf_counter()
                    plan.loglik(wss[w], olocs, oz, thetas[args.warmup + k], tol, out=o)
                    stream.synchronize()
                    clat[k] = time.perf_counter() - t0
                    cll[k] = o[2].item()

        torch.cuda.synchronize()
        t0 = time.perf_counter()
        threads = [threading.Thread(target=worker, args=(w,)) for w in range(conc)]
        for t in threads:
            t.start()
        for t in threads:
            t.join()
        torch.cuda.synchronize()
        ctotal = time.perf_counter() - t0
        cl = np.asarray(clat) * 1e3
        concurrent = {"evals_per_s": args.steps / ctotal, "streams": conc,
                      "latency_ms": {"p50": float(np.percentile(cl, 50)), "p99": float(np.percentile(cl, 99))},
                      "bitwise_equal_to_sequential": bool(all(a == b for a, b in zip(lls, cll)))}
        print(f"# {conc} in flight: {concurrent['evals_per_s']:.3f} evals/s", file=sys.stderr, flush=True)
    for k in stats[:3]:
        print(f"# timed {k['name']:20s} launches {k['launches']:7d}  total {k['total_ms']:10.2f} ms  "
              f"avg {1e3 * k['total_ms'] / max(k['launches'], 1):9.2f} us", file=sys.stderr)
    st = plan.status(ws)
    lat_ms = np.asarray(lat) * 1e3
    workload = (f"{args.config}: n={n} jittered grid, nu=0.5 beta=0.1 sigma2=1, {kind} order, nb={nb}, "
                f"tol={tol:g}, theta=theta_true*exp(0.2 N(0,I)) per step")
    rec = {
        "metric": "l(theta) evals/s, n=90k TLR Matern",
        "value": args.steps / total,
        "unit": "evals/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": 1e3 * total / args.steps,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n": n, "nb": nb, "tol": tol, "ordering": kind, "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "concurrent": concurrent,
        "max_rank": st["max_rank"],
        "rank_sum": st["rank_sum"],
        "all_finite": bool(np.all(np.isfinite(lls))),
        "roofline": roofline(stats, workload, warm_stats),
        # the same record for the busiest matrix-core GEMM class, from the
        # warm-up steps (where every class is timed): context for the above
        "roofline_gemm": next((roofline([w], workload, warm_stats) for w in warm_stats
                               if w["name"].startswith("k_gemm") and w["exact_launches"] > 0), None),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        ol = olocs.cpu().numpy()
        ozz = oz.cpu().numpy()
        rec["cpu_baseline"] = cpu_baseline(ol, ozz, theta_true, n, min(args.cpu_sample, n))
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
