"""HBM traffic per kernel launch from rocprofv3 counter passes.

Two counter passes of the same command -- one collecting FETCH_SIZE, one
WRITE_SIZE (KiB per dispatch) -- are reduced to mean KiB per launch for
every kernel.  The command also runs one plain device-to-device copy of a
known size (``bench.py --copy-probe-mib``); the ratio of its known bytes to
what the counters report for it calibrates the counters, and that factor
scales every kernel's figure.

    python -m paper_2402_09356_amd.traffic --fetch DIR --write DIR \\
        --copy-mib 1024 --workload "..." --out profiles/traffic.json

With --mfma DIR instead, it summarises a pass of the FP64 matrix-core
counters per kernel (flops per launch and busy share).
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
CSRC = os.path.join(ROOT, "paper_2402_09356_amd", "csrc")


def source_digest() -> str:
    h = hashlib.sha256()
    for f in sorted(os.listdir(CSRC)):
        if f.endswith((".hip", ".cpp", ".h")):
            with open(os.path.join(CSRC, f), "rb") as fh:
                h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


# kernel templates whose arguments name distinct timer classes; any other
# template's arguments are dropped (k_gen_tiles<0> -> k_gen_tiles)
_KEEP_ARGS = ("k_gemm_f64", "k_gemm_lds", "k_qrcp_regs")


def short_name(kernel: str) -> str:
    """Kernel class name as the launch timer reports it, from a mangled or
    demangled symbol: "k_gemm_f64<T,N>", "k_gemm_lds<N,N,64,32>",
    "k_qrcp_regs<8,6,12>", "k_chol_small", ..."""
    m = re.search(r"(k_[a-z][a-z_0-9]*?)I((?:L[bi]\d+E)+)([df]*)E", kernel)  # mangled template
    if m:
        base = m.group(1)
        args = re.findall(r"L([bi])(\d+)E", m.group(2))
        vals = [("T" if v == "1" else "N") if t == "b" else v for t, v in args]
        if m.group(3):
            vals.append(m.group(3))  # operand element types, e.g. "ddd" or "ffd"
    else:
        m = re.search(r"(k_[a-z][a-z_0-9]*)<([^>]*)>", kernel)  # demangled template
        if m:
            base = m.group(1)
            vals = []
            types = ""
            for a in m.group(2).split(","):
                a = a.strip()
                if a in ("double", "float"):
                    types += a[0]
                else:
                    vals.append({"true": "T", "false": "N"}.get(a, a))
            if types:
                vals.append(types)
        else:
            m = re.search(r"(k_[a-z][a-z_0-9]*)", kernel)
            return m.group(1) if m else kernel.split("(")[0][:60]
    if base not in _KEEP_ARGS:
        return base
    if base == "k_gemm_f64":
        vals = vals[:2]  # the wave count is not part of the timer class
    return "%s<%s>" % (base, ",".join(vals))


def read_counter(dirpath: str, counter: str):
    """{kernel name: [value per dispatch]} for one counter."""
    files = glob.glob(os.path.join(dirpath, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {dirpath}")
    per = defaultdict(dict)
    for f in files:
        with open(f, newline="") as fh:
            for row in csv.DictReader(fh):
                if row.get("Counter_Name") != counter:
                    continue
                key = (f, row.get("Dispatch_Id") or row.get("Correlation_Id"))
                per[row["Kernel_Name"]][key] = per[row["Kernel_Name"]].get(key, 0.0) + float(row["Counter_Value"])
    return {k: list(v.values()) for k, v in per.items()}


def mfma_summary(dirpath: str, simds: int = 1024) -> dict:
    """Per kernel class: FP64 matrix-core flops per launch (SQ_INSTS_VALU_MFMA_MOPS_F64
    counts 512 flops a unit) and the share of SIMD cycles the matrix cores were busy
    while the kernel ran (SQ_VALU_MFMA_BUSY_CYCLES over GRBM_GUI_ACTIVE x SIMDs)."""
    mops = read_counter(dirpath, "SQ_INSTS_VALU_MFMA_MOPS_F64")
    busy = read_counter(dirpath, "SQ_VALU_MFMA_BUSY_CYCLES")
    active = read_counter(dirpath, "GRBM_GUI_ACTIVE")
    out = {}
    for k in mops:
        name = short_name(k)
        if not name.startswith("k_"):
            continue
        rec = out.setdefault(name, {"dispatches": 0, "mfma_f64_flops": 0.0, "busy": 0.0, "active": 0.0})
        rec["dispatches"] += len(mops[k])
        rec["mfma_f64_flops"] += 512.0 * sum(mops[k])
        rec["busy"] += sum(busy.get(k, []))
        rec["active"] += sum(active.get(k, []))
    for rec in out.values():
        rec["mfma_f64_flops_per_launch"] = rec["mfma_f64_flops"] / max(rec["dispatches"], 1)
        rec["mfma_busy_frac"] = rec["busy"] / (rec["active"] * simds) if rec["active"] > 0 else None
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--fetch")
    ap.add_argument("--write")
    ap.add_argument("--copy-mib", type=float)
    ap.add_argument("--workload", required=True)
    ap.add_argument("--command", required=True, help="command line the passes profiled")
    ap.add_argument("--out", required=True)
    ap.add_argument("--mfma", help="directory of a SQ_INSTS_VALU_MFMA_MOPS_F64 / SQ_VALU_MFMA_BUSY_CYCLES / "
                                   "GRBM_GUI_ACTIVE pass: write its per-kernel summary instead")
    args = ap.parse_args()
    if args.mfma:
        rec = {"workload": args.workload, "source_sha256": source_digest(), "command": args.command,
               "kernels": mfma_summary(args.mfma)}
        with open(args.out, "w") as fh:
            json.dump(rec, fh, indent=1)
        print(json.dumps({"kernels": len(rec["kernels"])}))
        return
    fetch = read_counter(args.fetch, "FETCH_SIZE")
    write = read_counter(args.write, "WRITE_SIZE")
    copy_bytes = args.copy_mib * 2**20
    copy_names = [k for k in fetch if "copy" in k.lower() or "elementwise" in k.lower()]
    # the probe is the one copy dispatch whose fetch is closest to its size
    best = None
    for k in copy_names:
        for v in fetch[k]:
            if best is None or abs(v * 1024 - copy_bytes) < abs(best[1] * 1024 - copy_bytes):
                best = (k, v)
    if best is None:
        raise SystemExit("copy probe not found in the FETCH_SIZE pass")
    wbest = min((v for v in write.get(best[0], [])), key=lambda v: abs(v * 1024 - copy_bytes), default=None)
    f_fetch = copy_bytes / (best[1] * 1024)
    f_write = copy_bytes / (wbest * 1024) if wbest else None
    kernels = {}
    for k, vals in fetch.items():
        name = short_name(k)
        if name in kernels or not name.startswith("k_"):
            continue
        fv = [v for kk, vv in fetch.items() if short_name(kk) == name for v in vv]
        wv = [v for kk, vv in write.items() if short_name(kk) == name for v in vv]
        mf = sum(fv) / len(fv) * 1024 * f_fetch
        mw = (sum(wv) / len(wv) * 1024 * f_write) if (wv and f_write) else 0.0
        kernels[name] = {"dispatches": len(fv), "fetch_bytes_per_launch": mf, "write_bytes_per_launch": mw,
                         "hbm_bytes_per_launch": mf + mw}
    rec = {"workload": args.workload, "source_sha256": source_digest(), "command": args.command,
           "copy_probe": {"kernel": best[0][:80], "bytes": copy_bytes, "fetch_kib": best[1], "write_kib": wbest,
                          "fetch_factor": f_fetch, "write_factor": f_write},
           "kernels": kernels}
    with open(args.out, "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps({"copy_probe": rec["copy_probe"], "kernels": len(kernels)}))


if __name__ == "__main__":
    main()
