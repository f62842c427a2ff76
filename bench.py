"""Throughput of l(theta) evaluations through the TLR path on one MI355X.

Workload (default): n = 90,000 locations on a 300 x 300 jittered grid in the
unit square, Matern nu = 1/2, beta = 0.1, sigma2 = 1, Hilbert ordering, tiles
of nb = 900 (100 x 100 tiles), accuracy threshold tol = 1e-7.  The
observations Z ~ N(0, Sigma(theta_true)) are the stored draw of the blocked
dense oracle (tests/golden/large_c3_z.npy).  One step is one full evaluation:
covariance generation, per-tile compression, TLR Cholesky, forward solve,
log-determinant and l, at parameters theta_true * exp(0.2 N(0,I)) (seeded; a
fresh theta every step, as an optimiser would propose).  Inputs (ordered
locations, observations) are resident in HBM before timing starts.

`value` is evaluations per second with one evaluation at a time (the timed
steps, where the launch timer measures the dominant kernel on its stream).
After the timed steps:
  * accuracy: l at every theta the oracle stored for this workload, against
    the oracle's value (|dl| and |dl|/n);
  * roofline_eval: the whole evaluation at theta_true against the sum over
    its phases of max(flops / peak, bytes / peak), counted from that
    evaluation's own rank tables, with measured and published peaks;
  * concurrent: the same steps with three evaluations in flight, each on its
    own stream and workspace (bitwise check against one at a time).

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
    # name: (grid m, nb, tol, theta_true, ordering, config number for seeds, stored oracle values)
    "c1": (40, 200, 1e-9, (1.0, 0.1, 0.5), "morton", 1, "c1"),
    "c3": (300, 900, 1e-7, (1.0, 0.1, 0.5), "hilbert", 3, "c3"),
}
GOLDEN = os.path.join(ROOT, "tests", "golden")


def _cores():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count()
    return min(cores, int(os.environ.get("OMP_NUM_THREADS", cores)))


def cpu_baseline(locs_ordered: np.ndarray, z_ordered: np.ndarray, theta, n_full: int, sample_n: int,
                 full: bool = False):
    """The dense oracle timed on this host.  `value`: l on the first sample_n
    ordered points, extrapolated to n_full by n^3.  Also timed outright:
    n = 1,600 on one thread and on every core, and with full=True n = 40,000
    by the blocked oracle (all cores)."""
    import oracle.likelihood as OL

    sub_l, sub_z = locs_ordered[:sample_n], z_ordered[:sample_n]
    t0 = time.perf_counter()
    OL.loglik_dense(sub_l, sub_z, theta)
    dt = time.perf_counter() - t0
    scale = (n_full / sample_n) ** 3
    cores = _cores()
    measured = {}
    import synthetic

    small = synthetic.jittered_grid(40, synthetic.seed_for(1, synthetic.SEED_LOCS))
    zs = synthetic.standard_normal(1600, synthetic.seed_for(1, synthetic.SEED_Z))
    try:
        from threadpoolctl import threadpool_limits
    except ImportError:
        threadpool_limits = None
    OL.loglik_dense(small, zs, theta)
    t0 = time.perf_counter()
    OL.loglik_dense(small, zs, theta)
    measured["n1600_all_cores_s"] = time.perf_counter() - t0
    if threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            OL.loglik_dense(small, zs, theta)
            measured["n1600_one_thread_s"] = time.perf_counter() - t0
    if full:
        import oracle.blocked as OB

        big = synthetic.jittered_grid(200, synthetic.seed_for(2, synthetic.SEED_LOCS, 1))
        zb = synthetic.standard_normal(40000, synthetic.seed_for(2, synthetic.SEED_Z, 1))
        t0 = time.perf_counter()
        OB.loglik_blocked(big, zb, theta, b=4000)
        measured["n40000_all_cores_s"] = time.perf_counter() - t0
    return {"value": 1.0 / (dt * scale), "unit": "evals/s", "cores": cores, "kind": "oracle",
            "sample": f"dense float64 oracle l (Matern matrix, LAPACK Cholesky, solve) on the first {sample_n} "
                      f"ordered points: {dt:.2f} s; evals/s extrapolated to n={n_full} by (n/{sample_n})^3",
            "measured": measured}


# MI355X published peaks used for roofline fractions
PEAK_HBM_GBS = 8000.0
PEAK_FP64_TFLOPS = 78.6      # FP64 matrix (MFMA) and FP64 vector alike
VALU_KERNELS = ("k_chol_small", "k_trsm_rows", "k_qrcp_trunc", "k_qrcp_reg", "k_jacobi_svd",
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
    ap.add_argument("--precision", default="fp64", choices=["fp64", "mixed"],
                    help="mixed: low-rank factors stored in float32 (float64 arithmetic, diagonal tiles, "
                         "log-determinant and quadratic form)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-sample", type=int, default=10000)
    ap.add_argument("--cpu-full", action="store_true", help="also time the blocked oracle at n = 40,000")
    ap.add_argument("--no-peaks", action="store_true", help="skip the measured-peak probes")
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
    from paper_2402_09356_amd import roofline as RF

    if not torch.cuda.is_available():
        raise RuntimeError("bench.py needs a GPU")
    dev = torch.device("cuda:0")
    m, nb, tol, theta_true, kind, cfg, gname = CONFIGS[args.config]
    n = m * m
    locs = synthetic.jittered_grid(m, synthetic.seed_for(cfg, synthetic.SEED_LOCS))
    # Z ~ N(0, Sigma(theta_true)): the blocked dense oracle's stored draw
    with open(os.path.join(GOLDEN, f"large_{gname}.json")) as fh:
        golden = json.load(fh)
    z = np.load(os.path.join(GOLDEN, golden["z_file"]))
    if z.size != n or golden["seed_locs"] != synthetic.seed_for(cfg, synthetic.SEED_LOCS):
        raise RuntimeError("stored observations do not belong to this workload")
    thetas = synthetic.theta_perturbations(theta_true, args.warmup + args.steps,
                                           synthetic.seed_for(cfg, synthetic.SEED_THETA))

    dlocs = torch.from_numpy(locs).to(dev)
    perm = B.reorder(dlocs, kind, synthetic.seed_for(cfg, synthetic.SEED_ORDER))
    olocs, oz = B.apply_perm(perm, dlocs, torch.from_numpy(z).to(dev))
    plan = B.Plan(n, nb, precision={"fp64": "fp64", "mixed": "mixed_fp32"}[args.precision])
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

    # accuracy at every stored theta; the first (theta_true) also gives the
    # rank tables and the time for the whole-evaluation roofline
    acc_vals = []
    eval_ms = None
    rsig = rL = None
    for v in golden["values"]:
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        plan.loglik(ws, olocs, oz, tuple(v["theta"]), tol, out=out)
        torch.cuda.synchronize()
        dt_ms = 1e3 * (time.perf_counter() - t0)
        got = out.cpu().numpy()
        if eval_ms is None:
            eval_ms = dt_ms
            rsig, rL = plan.ranks(ws), plan.ranks(ws, factor=True)
        dl = abs(float(got[2]) - v["loglik"])
        acc_vals.append({"theta": v["theta"], "l_gpu": float(got[2]), "l_oracle": v["loglik"], "abs_dl": dl,
                         "abs_dl_per_n": dl / n, "abs_dlogdet": abs(float(got[0]) - v["logdet"]), "ms": dt_ms})
        print(f"# accuracy theta={v['theta']}: gpu {got[2]!r} oracle {v['loglik']!r} |dl|={dl:.3e}",
              file=sys.stderr, flush=True)
    # rank tables of the last stored theta's evaluation (read before the
    # concurrency run below evaluates other thetas on this workspace)
    st = plan.status(ws)
    bound_per_n = 1e-8 if args.precision == "fp64" else 1e-6
    accuracy = {"values": acc_vals, "max_abs_dl": max(a["abs_dl"] for a in acc_vals),
                "bound_per_n": bound_per_n,
                "within_bound": all(a["abs_dl_per_n"] <= bound_per_n for a in acc_vals),
                "oracle": "blocked dense FP64 Cholesky of Sigma(theta), stored in tests/golden"}

    peaks = {"hbm_gbs_spec": PEAK_HBM_GBS, "fp64_tflops_spec": PEAK_FP64_TFLOPS}
    if not args.no_peaks:
        peaks["hbm_gbs_measured"] = B.peak_hbm(4.0, 10, dev)
        peaks["fp64_tflops_measured"] = B.peak_mfma_f64(20000, dev)
        torch.cuda.synchronize()
        print(f"# measured peaks: HBM {peaks['hbm_gbs_measured']:.0f} GB/s, FP64 MFMA "
              f"{peaks['fp64_tflops_measured']:.1f} TFLOP/s", file=sys.stderr, flush=True)
    word = 8 if args.precision == "fp64" else 4
    work = RF.phase_work(n, nb, rsig, rL, factor_word=word)
    reval = {"spec": RF.roofline_eval(work, eval_ms, PEAK_FP64_TFLOPS, PEAK_HBM_GBS),
             "theta": list(theta_true), "factor_word_bytes": word}
    if "hbm_gbs_measured" in peaks:
        reval["measured_peaks"] = RF.roofline_eval(work, eval_ms, peaks["fp64_tflops_measured"],
                                                   peaks["hbm_gbs_measured"])
    reval["frac"] = reval.get("measured_peaks", reval["spec"])["frac"]

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
    lat_ms = np.asarray(lat) * 1e3
    workload = (f"{args.config}: n={n} jittered grid, nu=0.5 beta=0.1 sigma2=1, {kind} order, nb={nb}, "
                f"tol={tol:g}, theta=theta_true*exp(0.2 N(0,I)) per step, {args.precision}")
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
        "dtype": "f64" if args.precision == "fp64" else "f64/f32",
        "data": "synthetic",
        "config": {"workload": workload,
                   "n": n, "nb": nb, "tol": tol, "ordering": kind, "precision": args.precision},
        "latency_ms": {"p50": float(np.percentile(lat_ms, 50)), "p99": float(np.percentile(lat_ms, 99))},
        "accuracy": accuracy,
        "concurrent": concurrent,
        "max_rank": st["max_rank"],
        "rank_sum": st["rank_sum"],
        "all_finite": bool(np.all(np.isfinite(lls))),
        "roofline": roofline(stats, workload, warm_stats),
        "roofline_eval": reval,
        "peaks": peaks,
        # the same record for the busiest matrix-core GEMM class, from the
        # warm-up steps (where every class is timed): context for the above
        "roofline_gemm": next((roofline([w], workload, warm_stats) for w in warm_stats
                               if w["name"].startswith("k_gemm") and w["exact_launches"] > 0), None),
        "cpu_baseline": None,
    }
    if not args.no_cpu_baseline:
        ol = olocs.cpu().numpy()
        ozz = oz.cpu().numpy()
        rec["cpu_baseline"] = cpu_baseline(ol, ozz, theta_true, n, min(args.cpu_sample, n), args.cpu_full)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
