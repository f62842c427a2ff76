"""Write the large-n expected values: Z ~ N(0, Sigma(theta_true)) and l(theta).

Calls only the CPU oracle (the blocked dense Cholesky of ``oracle.blocked``)
and the seeded input generators; nothing here touches the GPU library.

Workloads (jittered m x m grid on the unit square, sigma2 = 1):

* ``c1``: m = 40 (n = 1,600), nu = 1/2, beta = 0.1 -- the small smoke case;
* ``c3``: m = 300 (n = 90,000), nu = 1/2, beta = 0.1 -- the n = 90,000 point of
  the paper's Section 5.3.1 timing study;
* ``c5-10k``: m = 100 (n = 10,000), nu = 1/2, beta = 0.1 -- the 10k problems of
  the serving workload;
* ``c2-<cell>``: m = 200 (n = 40,000), one (nu, beta) cell of the grid
  nu in {1/2, 3/2} x beta in {0.03, 0.1, 0.3} (cell = 3 * i_nu + i_beta).

For each workload Z = L e with L the lower Cholesky factor of Sigma(theta_true)
in generation order and e the seeded white noise; l(theta_true) then comes
from the same factor.  Further theta values (``--theta``) each take one more
blocked factorisation.  Output: ``large_<name>.json`` (the values) and
``large_<name>_z.npy`` (Z in generation order) beside this script.

    python tests/golden/make_large_golden.py --workload c3 --scratch DIR [--theta 1.2,0.08,0.5]

DIR receives the memory-mapped blocks (32 GB at n = 90,000) and is cleaned up.
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(os.path.dirname(HERE))
sys.path.insert(0, ROOT)

import synthetic  # noqa: E402
from oracle import blocked as OB  # noqa: E402

C2_CELLS = [(nu, beta) for nu in (0.5, 1.5) for beta in (0.03, 0.1, 0.3)]


def workload(name: str):
    if name == "c1":
        return dict(config=1, extra=0, m=40, theta=(1.0, 0.1, 0.5))
    if name == "c3":
        return dict(config=3, extra=0, m=300, theta=(1.0, 0.1, 0.5))
    if name == "c5-10k":
        return dict(config=5, extra=0, m=100, theta=(1.0, 0.1, 0.5))
    if name.startswith("c2-"):
        cell = int(name[3:])
        nu, beta = C2_CELLS[cell]
        return dict(config=2, extra=cell, m=200, theta=(1.0, beta, nu))
    raise ValueError(name)


def paths(name: str):
    return os.path.join(HERE, f"large_{name}.json"), os.path.join(HERE, f"large_{name}_z.npy")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--workload", required=True)
    ap.add_argument("--scratch", required=True)
    ap.add_argument("--block", type=int, default=4500)
    ap.add_argument("--theta", action="append", default=[], help="extra sigma2,beta,nu")
    args = ap.parse_args()
    w = workload(args.workload)
    jpath, zpath = paths(args.workload)
    os.makedirs(args.scratch, exist_ok=True)
    seed_locs = synthetic.seed_for(w["config"], synthetic.SEED_LOCS, w["extra"])
    seed_e = synthetic.seed_for(w["config"], synthetic.SEED_Z, w["extra"])
    locs = synthetic.jittered_grid(w["m"], seed_locs)
    n = locs.shape[0]
    log = lambda s: print(f"[{time.strftime('%H:%M:%S')}] {s}", flush=True)  # noqa: E731

    if os.path.exists(jpath) and os.path.exists(zpath):
        rec = json.load(open(jpath))
        z = np.load(zpath)
        log(f"extending {jpath}")
    else:
        e = synthetic.standard_normal(n, seed_e)
        t0 = time.time()
        f = OB.BlockedCholesky(locs, w["theta"], args.block, os.path.join(args.scratch, "blocks.bin"), log)
        t_fac = time.time() - t0
        z = f.matvec(e)
        res = f.loglik(z)
        f.close()
        np.save(zpath, z)
        rec = {
            "workload": args.workload,
            "n": n, "m": w["m"], "theta_true": list(w["theta"]),
            "seed_locs": seed_locs, "seed_e": seed_e, "block": args.block,
            "z_file": os.path.basename(zpath),
            "z_sha256": hashlib.sha256(np.ascontiguousarray(z).tobytes()).hexdigest(),
            "values": [{"theta": list(w["theta"]), "loglik": res.loglik, "logdet": res.logdet, "quad": res.quad,
                        "factor_seconds": t_fac}],
        }
        json.dump(rec, open(jpath, "w"), indent=1)
        log(f"l(theta_true) = {res.loglik!r} (factor {t_fac:.0f} s)")
    for spec in args.theta:
        th = tuple(float(v) for v in spec.split(","))
        if any(np.allclose(v["theta"], th, rtol=0, atol=0) for v in rec["values"]):
            continue
        t0 = time.time()
        f = OB.BlockedCholesky(locs, th, args.block, os.path.join(args.scratch, "blocks.bin"), log)
        res = f.loglik(z)
        f.close()
        rec["values"].append({"theta": list(th), "loglik": res.loglik, "logdet": res.logdet, "quad": res.quad,
                              "factor_seconds": time.time() - t0})
        json.dump(rec, open(jpath, "w"), indent=1)
        log(f"l{th} = {res.loglik!r}")


if __name__ == "__main__":
    main()
