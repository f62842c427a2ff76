"""Whole-evaluation roofline of one l(theta) evaluation.

The algorithmic work of each phase is counted from the evaluation's own rank
tables (the ranks of Sigma's compressed tiles and of the factor's tiles), as
the operations the method needs and each operand read and each result written
once in HBM -- not what this implementation happens to do:

* gen_tiles: every stored entry of Sigma (the nt diagonal tiles and the
  lower off-diagonal tiles) evaluated once (about 30 FP64 operations an entry
  for nu = 1/2) and written once, the off-diagonal ones read back once by the
  compression;
* compress: two sketch passes of 2 nb^2 (r + p) flops per tile (p = 8) and
  the factors U, V written (2 nb r words);
* tlr_potrf: dense Cholesky of the nt diagonal tiles (nb^3 / 3 each), the
  TRSM of every panel factor (nb^2 r), the symmetric update of every
  diagonal tile by each tile left of it (2 nb^2 r) and, for every i > j > k,
  the low-rank update of tile (i, j) by tiles (i, k), (j, k) with its
  recompression: 4 nb r_ik r_jk + 2 (4 nb s^2 - 4 s^3 / 3) + 22 s^3 +
  4 nb s r_ij flops with s = r_ij + r_jk, reading six factor panels and
  writing two;
* solve_logdet: the factors and the lower diagonal tiles read once, 4 flops
  per factor entry pair.

T_roof = sum over phases of max(F / P_flops, B / P_bytes); the fraction
reported is T_roof / T_measured.
"""
from __future__ import annotations

import numpy as np

MATERN_OPS_PER_ENTRY = 30.0
OVERSAMPLE = 8


def _lower(r):
    r = np.asarray(r, dtype=np.float64)
    nt = r.shape[0]
    il = np.tril_indices(nt, -1)
    out = np.zeros_like(r)
    out[il] = np.maximum(r[il], 0.0)
    return out


def phase_work(n: int, nb: int, rsig, rL, factor_word: int = 8) -> dict:
    """{phase: (flops, bytes)} of one evaluation; ranks are nt x nt tables
    (entries i > j used; negative entries, such as dense markers, count 0)."""
    nt = (n + nb - 1) // nb
    rs, rl = _lower(rsig), _lower(rL)
    ntiles = nt * (nt - 1) // 2
    entries = nt * nb * nb + ntiles * nb * nb
    gen = (MATERN_OPS_PER_ENTRY * entries, 8.0 * entries + 8.0 * ntiles * nb * nb)
    comp = (2.0 * 2.0 * nb * nb * (rs.sum() + OVERSAMPLE * ntiles), float(factor_word * 2.0 * nb * rs.sum()))
    f = nt * nb ** 3 / 3.0 + nb * nb * rl.sum() + 2.0 * nb * nb * rl.sum()
    b = 2.0 * 8.0 * nt * nb * nb
    for j in range(nt):
        for k in range(j):
            rjk = rl[j, k]
            if rjk <= 0:
                continue
            rik = rl[j + 1:, k]
            rij = rl[j + 1:, j]
            s = rij + rjk
            f += float(np.sum(4.0 * nb * rik * rjk + 2.0 * (4.0 * nb * s * s - 4.0 * s ** 3 / 3.0) + 22.0 * s ** 3
                              + 4.0 * nb * s * rij))
            b += float(np.sum(factor_word * nb * (2.0 * rik + 2.0 * rjk + 4.0 * rij)))
    pot = (f, b)
    sol = (4.0 * nb * rl.sum() + nt * nb * nb, factor_word * 2.0 * nb * rl.sum() + 8.0 * nt * nb * nb / 2.0
           + 16.0 * n)
    return {"gen_tiles": gen, "compress": comp, "tlr_potrf": pot, "solve_logdet": sol}


def roofline_eval(work: dict, t_measured_ms: float, peak_flops_tf: float, peak_gbs: float) -> dict:
    phases = {}
    t_roof = 0.0
    for name, (fl, by) in work.items():
        tf = fl / (peak_flops_tf * 1e12)
        tb = by / (peak_gbs * 1e9)
        t = max(tf, tb)
        t_roof += t
        phases[name] = {"flops": fl, "bytes": by, "t_roof_ms": 1e3 * t, "bound": "hbm" if tb >= tf else "fp64"}
    return {"t_roof_ms": 1e3 * t_roof, "t_measured_ms": t_measured_ms, "frac": 1e3 * t_roof / t_measured_ms,
            "peak_fp64_tflops": peak_flops_tf, "peak_hbm_gbs": peak_gbs, "phases": phases}
