"""Parity of the exact code path the n = 90,000 benchmark times.

The benchmark runs nb = 900 tiles with the default (pivoted-QR) truncation
and no rank request.  These tests run that path at sizes the dense oracle
finishes in seconds (n = 8,100 and a ragged n = 16,129), through the tall
LDS-staged GEMM kernels (checked directly against NumPy as well), the
global-memory pivoted QR and row TRSM for sketches wider than 192 columns,
and against the blocked dense oracle's stored values at n = 40,000 and
n = 90,000.

Bound for FP64 TLR at threshold tol: |l_TLR - l_dense| <= n max(1e-8, 0.1 tol)
(the compression-alone term of the small-n tests is below this for every
well-conditioned case here, so it is left out, which only tightens the test).
"""
import json
import os

import numpy as np
import pytest
import torch

import synthetic
from oracle import likelihood as OL
from oracle import ordering as OO
from oracle import tlr as OT
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")


def fp64_bound(n, tol):
    return n * max(1e-8, 0.1 * tol)


def grid_problem(m, theta, kind="hilbert", cfg=3, extra=7):
    locs = synthetic.jittered_grid(m, synthetic.seed_for(cfg, synthetic.SEED_LOCS, extra))
    n = locs.shape[0]
    e = synthetic.standard_normal(n, synthetic.seed_for(cfg, synthetic.SEED_Z, extra))
    z = OL.sample_field(locs, theta, e)
    perm = OO.reorder(locs, kind)
    return locs[perm], z[perm]


@pytest.mark.parametrize("trans_a,M,N,K,count,cls", [
    (False, 2048, 48, 900, 8, "k_gemm_lds<N,N>"),   # 64 x 64 blocks
    (False, 2000, 24, 900, 9, "k_gemm_lds<N,N>"),   # 64 x 32 blocks, ragged M
    (True, 1024, 100, 900, 16, "k_gemm_lds<T,N>"),  # 64 x 64 blocks
    (True, 1000, 20, 901, 17, "k_gemm_lds<T,N>"),   # 64 x 32 blocks, ragged M and K
])
def test_tall_gemm_kernels_against_numpy(trans_a, M, N, K, count, cls):
    device()
    rng = np.random.default_rng(M + N + K)
    a = rng.standard_normal((count, M, K) if trans_a else (count, K, M))
    b = rng.standard_normal((count, N, K))
    c0 = rng.standard_normal((count, N, M))
    da, db, dc = to_dev(a), to_dev(b), to_dev(c0)
    B.kstats_enable(True)
    B.kstats_reset()
    try:
        B.diag_gemm_strided(da, db, dc, trans_a=trans_a, alpha=-0.5, beta=2.0)
        torch.cuda.synchronize()
        st = {k["name"]: k["launches"] for k in B.kstats()}
    finally:
        B.kstats_enable(False)
    assert st.get(cls, 0) == 1, st
    got = dc.cpu().numpy()
    for t in range(count):
        A = a[t] if trans_a else a[t].T          # op(A), M x K
        Bm = b[t].T                                # K x N
        ref = (-0.5 * A @ Bm + 2.0 * c0[t].T).T
        np.testing.assert_allclose(got[t], ref, rtol=1e-12, atol=1e-11 * np.sqrt(K))


@pytest.mark.parametrize("m,nu,tol", [
    (90, 0.5, 1e-7), (90, 0.5, 1e-9), (90, 0.56, 1e-7), (90, 0.56, 1e-9),
    (127, 0.5, 1e-7), (127, 0.5, 1e-9),
])
def test_nb900_pivoted_qr_path(m, nu, tol):
    """nb = 900, Hilbert, default truncation, no rank request: l within the
    bound of the dense oracle; every tile's rank at or a few above its exact
    singular-value rank (n = 8,100)."""
    device()
    theta, nb = (1.0, 0.1, nu), 900
    locs, z = grid_problem(m, theta)
    n = locs.shape[0]
    print(f"nb900 n={n} nu={nu} tol={tol}", flush=True)
    plan = B.Plan(n, nb)
    ws = plan.workspace()
    out = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    dense = OL.loglik_dense(locs, z, theta)
    err = abs(out[2] - dense.loglik)
    print(f"  gpu {out[2]!r} dense {dense.loglik!r} |dl|={err:.3e} bound={fp64_bound(n, tol):.3e}", flush=True)
    assert plan.status(ws)["code"] == 0
    assert err <= fp64_bound(n, tol)
    assert abs(out[0] - dense.logdet) <= fp64_bound(n, tol)
    if m == 90 and nu == 0.5:
        ranks = plan.ranks(ws)
        tiles = [(i, j) for i in range(plan.nt) for j in range(i)]
        tsvd = OT.tile_svd_from_locations(locs, theta, nb, tiles)
        oranks, onum = OT.tile_ranks(tsvd, tol, maxrank=plan.maxrank)
        for (i, j) in tiles:
            assert onum[i, j] <= ranks[i, j] <= onum[i, j] + 12, (i, j, ranks[i, j], onum[i, j])
        bins = (0, 1, 11, 26, 51, 101, 201, 10**9)
        h_gpu = OT.rank_stats(ranks, ranks, bins)["hist"]
        h_svd = OT.rank_stats(oranks, onum, bins)["hist"]
        print(f"  rank histogram bins {bins}: pivoted QR {h_gpu}, singular values {h_svd}", flush=True)


def test_wide_sketch_path_end_to_end():
    """beta = 0.3 at tol = 1e-9 with nb = 900: the nearest tiles need sketches
    wider than 192 columns, which run the global-memory pivoted QR and row
    TRSM; l stays within the bound of the dense oracle."""
    device()
    theta, nb, tol = (1.0, 0.3, 0.5), 900, 1e-9
    locs, z = grid_problem(90, theta, extra=8)
    n = locs.shape[0]
    plan = B.Plan(n, nb)
    ws = plan.workspace()
    B.kstats_enable(True)
    B.kstats_reset()
    try:
        out = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
        torch.cuda.synchronize()
        st = {k["name"]: k["launches"] for k in B.kstats()}
    finally:
        B.kstats_enable(False)
    dense = OL.loglik_dense(locs, z, theta).loglik
    print(f"wide: gpu {out[2]!r} dense {dense!r} launches qrcp_trunc={st.get('k_qrcp_trunc', 0)} "
          f"trsm_rows_wide={st.get('k_trsm_rows_wide', 0)}", flush=True)
    assert st.get("k_qrcp_trunc", 0) >= 1 and st.get("k_trsm_rows_wide", 0) >= 1, st
    assert abs(out[2] - dense) <= fp64_bound(n, tol)


def _golden(name):
    jp = os.path.join(GOLDEN, f"large_{name}.json")
    if not os.path.exists(jp):
        pytest.skip(f"no stored values for {name}")
    rec = json.load(open(jp))
    z = np.load(os.path.join(GOLDEN, rec["z_file"]))
    return rec, z


def _large_problem(rec, z):
    cfg = 3 if rec["workload"] == "c3" else 2
    extra = 0 if cfg == 3 else int(rec["workload"][3:])
    locs = synthetic.jittered_grid(rec["m"], synthetic.seed_for(cfg, synthetic.SEED_LOCS, extra))
    assert locs.shape[0] == rec["n"] == z.size
    dev = device()
    dl = torch.from_numpy(locs).to(dev)
    perm = B.reorder(dl, "hilbert")
    return B.apply_perm(perm, dl, torch.from_numpy(z).to(dev))


@pytest.mark.parametrize("name,nb,tol", [("c2-1", 800, 1e-7), ("c2-1", 800, 1e-9), ("c2-3", 800, 1e-7),
                                         ("c3", 900, 1e-7)])
def test_large_n_against_blocked_oracle(name, nb, tol):
    """n = 40,000 and n = 90,000 jittered grids, Hilbert order: l at every
    stored theta within the bound of the blocked dense oracle's value."""
    rec, z = _golden(name)
    ol, oz = _large_problem(rec, z)
    n = rec["n"]
    plan = B.Plan(n, nb)
    ws = plan.workspace()
    for v in rec["values"]:
        print(f"{name} nb={nb} tol={tol} theta={v['theta']}", flush=True)
        out = plan.loglik(ws, ol, oz, tuple(v["theta"]), tol).cpu().numpy()
        err = abs(out[2] - v["loglik"])
        print(f"  gpu {out[2]!r} oracle {v['loglik']!r} |dl|={err:.3e} |dl|/n={err / n:.2e}", flush=True)
        assert plan.status(ws)["code"] == 0
        assert err <= fp64_bound(n, tol)


def _compressed_cells():
    jp = os.path.join(GOLDEN, "compressed_c2.json")
    if not os.path.exists(jp):
        return []
    return [(r["cell"], r["nb"], r["tol"]) for r in json.load(open(jp)) if r["delta_c"] is not None]


@pytest.mark.parametrize("cell,nb,tol", _compressed_cells())
def test_smooth_cells_within_compression_bound(cell, nb, tol):
    """nu = 3/2 datasets at n = 40,000 (ill-conditioned): l within
    max(n max(1e-8, 0.1 tol), 10 |delta_c|), delta_c = l(Sigma~) - l(Sigma) from
    the tile-truncated blocked oracle with the same tiles (Hilbert order)."""
    rec = {(r["cell"], r["nb"], r["tol"]): r for r in json.load(open(os.path.join(GOLDEN, "compressed_c2.json")))}
    dc = rec[(cell, nb, tol)]["delta_c"]
    g, z = _golden(f"c2-{cell}")
    ol, oz = _large_problem(g, z)
    n = g["n"]
    plan = B.Plan(n, nb, maxrank=nb // 2, dense_tiles=True)
    ws = plan.workspace()
    out = plan.loglik(ws, ol, oz, tuple(g["theta_true"]), tol).cpu().numpy()
    err = abs(out[2] - g["values"][0]["loglik"])
    bnd = max(n * max(1e-8, 0.1 * tol), 10 * abs(dc))
    print(f"smooth cell {cell} nb={nb} tol={tol}: |dl|/n {err / n:.2e}, delta_c/n {dc / n:.2e}, "
          f"bound/n {bnd / n:.2e}", flush=True)
    assert plan.status(ws)["code"] == 0
    assert err <= bnd
