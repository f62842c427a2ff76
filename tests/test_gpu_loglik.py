"""End-to-end parity of the TLR likelihood path against the oracle.

Acceptance bound for FP64 TLR at threshold tol (compression error alone is
delta_c = l(Sigma~) - l(Sigma), from the oracle):
    |l_TLR - l_dense| <= max(n * max(1e-8, 0.1 * tol), 10 * |delta_c|)
and |l_TLR - l_dense| <= 1e-8 * n at tol = 1e-12.  The factor 10 covers the
single re-compression of each Schur-complement tile, which adds truncation
error of the same order as the initial compression.
"""
import numpy as np
import pytest
import torch

import synthetic
from oracle import likelihood as OL
from oracle import matern as OM
from oracle import ordering as OO
from oracle import tlr as OT
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, from_colmajor, to_dev

pytestmark = pytest.mark.gpu


def bound(n, tol, delta_c):
    return max(n * max(1e-8, 0.1 * tol), 10 * abs(delta_c))


def make_problem(m, theta, kind, cfg=1, locs=None):
    if locs is None:
        locs = synthetic.jittered_grid(m, synthetic.seed_for(cfg, synthetic.SEED_LOCS))
    n = locs.shape[0]
    e = synthetic.standard_normal(n, synthetic.seed_for(cfg, synthetic.SEED_Z))
    z = OL.sample_field(locs, theta, e)
    perm = OO.reorder(locs, kind, seed=synthetic.seed_for(cfg, synthetic.SEED_ORDER))
    return locs[perm], z[perm]


def run_gpu(locs, z, theta, nb, tol, maxrank=0, truncation="qrcp", precision="fp64"):
    plan = B.Plan(locs.shape[0], nb, maxrank=maxrank, truncation=truncation, precision=precision)
    ws = plan.workspace()
    dl, dz = to_dev(locs), to_dev(z)
    ranks = torch.zeros(plan.nt * plan.nt, dtype=torch.int32, device=dl.device)
    out = plan.loglik(ws, dl, dz, theta, tol, ranks=ranks)
    torch.cuda.synchronize()
    return plan, ws, out.cpu().numpy(), ranks.cpu().numpy().reshape(plan.nt, plan.nt)


def test_c1_smoke_configuration():
    """n=1,600 jittered grid, nu=1/2, beta=0.1, Morton, nb=200, tol=1e-9."""
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs, z = make_problem(40, theta, "morton")
    print("c1 loglik", flush=True)
    plan, ws, out, ranks = run_gpu(locs, z, theta, nb, tol)
    dense = OL.loglik_dense(locs, z, theta)
    comp, oranks = OT.compressed_loglik(locs, z, theta, nb, tol)
    delta_c = comp.loglik - dense.loglik
    err = abs(out[2] - dense.loglik)
    print(f"c1: gpu {out[2]!r} dense {dense.loglik!r} |d|={err:.3e} delta_c={delta_c:.3e}", flush=True)
    assert np.isfinite(out[2])
    assert err <= bound(1600, tol, delta_c)
    assert abs(out[0] - dense.logdet) <= bound(1600, tol, delta_c)
    # the workspace's rank tables: Sigma's equal what compress returned; L's lie in [0, maxrank]
    np.testing.assert_array_equal(plan.ranks(ws), ranks)
    lr = plan.ranks(ws, factor=True)
    low = lr[np.tril_indices(plan.nt, -1)]
    assert np.all((low >= 0) & (low <= plan.maxrank))
    # pivoted-QR ranks: at or a few above the exact SVD ranks
    sv = OT.tile_svd(OM.covariance_matrix(locs, theta), nb)
    for (i, j), s in sv.svals.items():
        exact = OT.numerical_rank(s, tol)
        assert exact <= ranks[i, j] <= exact + 12, (i, j, ranks[i, j], exact)
    # with the singular-value rule: equal to the exact SVD ranks except inside the tie band
    plan2, ws2, out2, ranks2 = run_gpu(locs, z, theta, nb, tol, truncation="svd")
    assert abs(out2[2] - dense.loglik) <= bound(1600, tol, delta_c)
    for (i, j), s in sv.svals.items():
        exact = OT.numerical_rank(s, tol)
        if ranks2[i, j] != exact:
            lo, hi = sorted((ranks2[i, j], exact))
            band = s[lo:hi + 1]
            assert hi - lo <= 1 and np.all(np.abs(band / tol - 1) < 1e-3), (i, j, ranks2[i, j], exact)


def test_compressed_tiles_and_diagonal_match_oracle():
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs, z = make_problem(40, theta, "hilbert")
    plan = B.Plan(1600, nb)
    ws = plan.workspace()
    plan.gen_tiles(ws, to_dev(locs), theta)
    sig = OM.covariance_matrix(locs, theta)
    for k in (0, 3, 7):
        tile, _ = plan.tile(ws, k, k)
        ref = sig[k * nb:(k + 1) * nb, k * nb:(k + 1) * nb]
        np.testing.assert_allclose(tile, ref, rtol=1e-14, atol=1e-300)
    plan.compress(ws, tol)
    for (i, j) in [(1, 0), (5, 2), (7, 6), (7, 0)]:
        tile, r = plan.tile(ws, i, j)
        ref = sig[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
        err = np.linalg.norm(tile - ref, 2)
        # pivoted-QR truncation: trailing Frobenius norm <= tol bounds the
        # spectral error; the rest is the rounding of the tile's own norm
        assert err <= 1.5 * tol + 1e-15 * np.linalg.norm(ref, 2), (i, j, r, err)


def test_tol_1e12_reaches_dense():
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 200, 1e-12
    locs, z = make_problem(40, theta, "morton")
    print("tol 1e-12", flush=True)
    plan, ws, out, ranks = run_gpu(locs, z, theta, nb, tol, maxrank=nb)
    dense = OL.loglik_dense(locs, z, theta).loglik
    print(f"tol12: gpu {out[2]!r} dense {dense!r}", flush=True)
    assert abs(out[2] - dense) <= 1e-8 * 1600


@pytest.mark.parametrize("kind", ["none", "random", "morton", "hilbert", "kdtree"])
def test_every_ordering_small(kind):
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 100, 1e-9
    locs, z = make_problem(30, theta, kind)
    n = locs.shape[0]
    print(f"ordering {kind}", flush=True)
    plan, ws, out, ranks = run_gpu(locs, z, theta, nb, tol, maxrank=nb)
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, _ = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=nb)
    assert abs(out[2] - dense) <= bound(n, tol, comp.loglik - dense)


@pytest.mark.parametrize("nu", [0.8, 1.0, 1.5, 2.5])
def test_general_smoothness(nu):
    device()
    theta, nb, tol = (1.3, 0.07, nu), 128, 1e-9
    locs, z = make_problem(30, theta, "hilbert")
    n = locs.shape[0]
    plan = B.Plan(n, nb)
    ws = plan.workspace()
    plan.gen_tiles(ws, to_dev(locs), theta)
    sig = OM.covariance_matrix(locs, theta)
    tile, _ = plan.tile(ws, 1, 1)
    ref = sig[nb:2 * nb, nb:2 * nb]
    np.testing.assert_allclose(tile, ref, rtol=2e-13, atol=1e-300)
    print(f"nu={nu}", flush=True)
    plan2, ws2, out, _ = run_gpu(locs, z, theta, nb, tol, maxrank=nb)
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, _ = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=nb)
    assert abs(out[2] - dense) <= bound(n, tol, comp.loglik - dense)


def test_ragged_tiles():
    device()
    theta, nb, tol = (1.0, 0.05, 0.5), 128, 1e-9
    locs = synthetic.uniform_points(1000, 77)
    locs, z = make_problem(0, theta, "kdtree", locs=locs)
    plan, ws, out, _ = run_gpu(locs, z, theta, nb, tol, maxrank=nb)
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, _ = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=nb)
    assert abs(out[2] - dense) <= bound(1000, tol, comp.loglik - dense)


def test_deterministic_repeat():
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs, z = make_problem(40, theta, "hilbert")
    plan = B.Plan(1600, nb)
    ws = plan.workspace()
    a = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    b = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    ws2 = plan.workspace()
    c = plan.loglik(ws2, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    # no state is carried between evaluations: bitwise identical results
    assert a.tobytes() == b.tobytes() == c.tobytes()


@pytest.mark.parametrize("theta", [(1.0, 0.1, 1.5), (1.0, 0.1, 0.5)])
def test_not_spd_agrees_with_oracle(theta):
    """Both sides fail a pivot that is not positive (LAPACK's rule).  Fifty
    duplicated locations make Sigma exactly singular fifty times over, so the
    computed pivots of the duplicates are rounding noise of either sign and
    at least one is not positive on both sides; the same points without the
    duplicates are SPD on both sides."""
    device()
    base = synthetic.uniform_points(300, 5)
    z = synthetic.standard_normal(300, 6)
    locs = base.copy()
    locs[150:200] = locs[:50]
    with pytest.raises(OL.NotPositiveDefinite):
        OL.loglik_dense(locs, z, theta)
    plan, ws, out, _ = run_gpu(locs, z, theta, 64, 1e-9, maxrank=64)
    assert out[2] == -np.inf
    assert plan.status(ws)["code"] == 16
    dense = OL.loglik_dense(base, z, theta).loglik
    plan, ws, out, _ = run_gpu(base, z, theta, 64, 1e-9, maxrank=64)
    assert plan.status(ws)["code"] == 0 and np.isfinite(out[2])
    comp, _ = OT.compressed_loglik(base, z, theta, 64, 1e-9, maxrank=64)
    assert abs(out[2] - dense) <= bound(300, 1e-9, comp.loglik - dense)


def test_rank_overflow_surfaces_as_minus_inf():
    device()
    locs2, z2 = make_problem(20, (1.0, 0.1, 0.5), "random")
    plan2, ws2, out2, ranks2 = run_gpu(locs2, z2, (1.0, 0.1, 0.5), 100, 1e-9, maxrank=2)
    assert out2[2] == -np.inf
    assert plan2.status(ws2)["code"] == 17
    assert (ranks2[np.tril_indices(4, -1)] == -1).any()


def test_collinear_ar1_exact_at_scale():
    """Points sorted along a line with nu = 1/2: exact l by the Markov
    factorisation, any n (here 20,000 with nb = 400)."""
    device()
    n, nb, tol = 20000, 400, 1e-12
    locs = synthetic.collinear_points(n, 8)
    sigma2, beta = 1.0, 0.02
    e = synthetic.standard_normal(n, 9)
    t = locs[:, 0] * np.sqrt(2.0)
    rho = np.exp(-np.diff(t) / beta)
    var = sigma2 * (1 - rho * rho)
    # an exact draw from the model by its Markov recursion
    z = np.empty(n)
    z[0] = np.sqrt(sigma2) * e[0]
    for k in range(1, n):
        z[k] = rho[k - 1] * z[k - 1] + np.sqrt(var[k - 1]) * e[k]
    r = z[1:] - rho * z[:-1]
    ref = (-0.5 * np.log(2 * np.pi) - 0.5 * np.log(sigma2) - z[0] ** 2 / (2 * sigma2)
           + np.sum(-0.5 * np.log(2 * np.pi) - 0.5 * np.log(var) - r * r / (2 * var)))
    print("ar1 20000", flush=True)
    plan, ws, out, ranks = run_gpu(locs, z, (sigma2, beta, 0.5), nb, tol)
    assert abs(out[2] - ref) <= 1e-8 * n
    # off-diagonal tiles of the exponential kernel on a sorted line have rank 1
    low = ranks[np.tril_indices(plan.nt, -1)]
    assert np.all(low <= 1)


@pytest.mark.parametrize("kind,tol,maxrank", [("morton", 1e-9, 0), ("hilbert", 1e-7, 0), ("kdtree", 1e-9, 0),
                                              ("morton", 1e-12, 200)])
def test_fast_truncation_path(kind, tol, maxrank):
    """Without a rank request the compression truncates by pivoted QR
    (trailing Frobenius norm <= tol): error per tile <= tol, l within bound.
    At tol = 1e-12 the ranks reach ~125, so the sketch widths exercise the
    wide (packed / register-resident) small kernels."""
    device()
    theta, nb = (1.0, 0.1, 0.5), 200
    locs, z = make_problem(40, theta, kind)
    plan = B.Plan(1600, nb, maxrank=maxrank)
    ws = plan.workspace()
    out = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, oranks = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=maxrank or None)
    assert abs(out[2] - dense) <= bound(1600, tol, comp.loglik - dense)
    plan.gen_tiles(ws, to_dev(locs), theta)
    plan.compress(ws, tol)
    sig = OM.covariance_matrix(locs, theta)
    for (i, j) in [(1, 0), (4, 3), (7, 2)]:
        tile, r = plan.tile(ws, i, j)
        ref = sig[i * nb:(i + 1) * nb, j * nb:(j + 1) * nb]
        assert np.linalg.norm(tile - ref, 2) <= 1.5 * tol + 1e-15 * np.linalg.norm(ref, 2)
        assert oranks[i, j] <= r <= oranks[i, j] + 12


@pytest.mark.parametrize("kind", ["random", "morton", "hilbert", "kdtree"])
def test_rank_histograms_match_oracle_per_ordering(kind):
    """Singular-value truncation at n = 6,400 (80 x 80 jittered grid), nb = 400,
    tol = 1e-7: every off-diagonal tile's rank equals the oracle's SVD rank
    except inside the singular-value tie band, and the rank histograms agree
    up to those tiles."""
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 400, 1e-7
    locs, z = make_problem(80, theta, kind, cfg=2)
    n = locs.shape[0]
    plan = B.Plan(n, nb, maxrank=nb, truncation="svd")
    ws = plan.workspace()
    ranks_dev = torch.empty((plan.nt, plan.nt), dtype=torch.int32, device="cuda")
    plan.gen_tiles(ws, to_dev(locs), theta)
    plan.compress(ws, tol, ranks=ranks_dev)
    ranks = ranks_dev.cpu().numpy()
    nt = plan.nt
    tiles = [(i, j) for i in range(nt) for j in range(i)]
    tsvd = OT.tile_svd_from_locations(locs, theta, nb, tiles)
    oranks, onum = OT.tile_ranks(tsvd, tol, maxrank=nb)
    ties = 0
    for (i, j) in tiles:
        if ranks[i, j] != oranks[i, j]:
            s = tsvd.svals[(i, j)]
            lo, hi = sorted((int(ranks[i, j]), int(oranks[i, j])))
            assert hi - lo <= 1 and np.all(np.abs(s[lo:hi + 1] / tol - 1) < 1e-3), (kind, i, j, ranks[i, j],
                                                                                      oranks[i, j])
            ties += 1
    gpu_ranks = oranks.copy()
    for (i, j) in tiles:
        gpu_ranks[i, j] = ranks[i, j]
    h_gpu = OT.rank_stats(gpu_ranks, gpu_ranks, bins=(0, 1, 11, 26, 51, 101, 201, 10**9))["hist"]
    h_ora = OT.rank_stats(oranks, onum, bins=(0, 1, 11, 26, 51, 101, 201, 10**9))["hist"]
    print(kind, "hist gpu", h_gpu, "oracle", h_ora, "tie tiles", ties, flush=True)
    assert sum(abs(a - b) for a, b in zip(h_gpu, h_ora)) <= 2 * ties


def test_dense_tile_fallback_matches_oracle():
    """maxrank = 48 with dense tiles allowed: every tile whose rank exceeds 48 is
    kept dense (compression and recompressions), as the oracle's tile-truncated
    matrix does; l agrees with the dense oracle within the bound, dense tiles
    read back as -2, and the evaluation is bitwise repeatable."""
    device()
    theta, nb, tol, cap = (1.0, 0.1, 0.5), 200, 1e-9, 48
    locs, z = make_problem(40, theta, "morton")
    plan = B.Plan(1600, nb, maxrank=cap, dense_tiles=True)
    ws = plan.workspace()
    dl, dz = to_dev(locs), to_dev(z)
    out = plan.loglik(ws, dl, dz, theta, tol).cpu().numpy()
    assert plan.status(ws)["code"] == 0
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, oranks = OT.compressed_loglik(locs, z, theta, nb, tol, maxrank=cap)
    print("dense fallback", out[2], dense, comp.loglik, flush=True)
    assert abs(out[2] - dense) <= bound(1600, tol, comp.loglik - dense)
    rk = plan.ranks(ws)
    low = np.tril_indices(plan.nt, -1)
    # every tile the oracle keeps dense is dense here (the pivoted-QR rank is >= the SVD rank)
    assert np.all(rk[low][oranks[low] == OT.DENSE] == -2)
    assert (rk[low] == -2).sum() >= 1 and (rk[low] >= 0).sum() >= 1
    out2 = plan.loglik(ws, dl, dz, theta, tol).cpu().numpy()
    assert out2[2] == out[2]


def test_dense_tiles_random_order():
    """Random order makes most tiles full rank at tol = 1e-9: with dense tiles
    the evaluation goes through and matches the dense oracle."""
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 100, 1e-9
    locs, z = make_problem(30, theta, "random")
    plan = B.Plan(900, nb, dense_tiles=True)
    ws = plan.workspace()
    out = plan.loglik(ws, to_dev(locs), to_dev(z), theta, tol).cpu().numpy()
    dense = OL.loglik_dense(locs, z, theta).loglik
    comp, _ = OT.compressed_loglik(locs, z, theta, nb, tol)
    assert plan.status(ws)["code"] == 0
    assert abs(out[2] - dense) <= bound(900, tol, comp.loglik - dense)
    assert (plan.ranks(ws)[np.tril_indices(plan.nt, -1)] == -2).sum() >= 1


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_evaluation_allocates_no_device_memory(precision):
    """The workspace is the only device memory an evaluation uses.  Once
    the library's pooled streams and pinned staging buffers exist (one pass
    over a sequence of evaluations), two more passes create none.  The
    device's free memory over those passes moves by at most the HIP
    runtime's own queue pools (kernel arguments, signals), which grow in
    2 MiB steps with the depth of queued work, a few steps at most; a
    device allocation of the library's (a workspace-sized buffer is
    hundreds of MB here) would exceed that."""
    import gc

    dev = device()
    theta, nb, tol = (1.0, 0.1, 0.5), 900, 1e-7
    locs = synthetic.jittered_grid(90, synthetic.seed_for(3, synthetic.SEED_LOCS, 7))
    z = synthetic.standard_normal(8100, 5)
    plan = B.Plan(8100, nb, precision=precision)
    ws = plan.workspace()
    dl, dz = to_dev(locs), to_dev(z)
    out = torch.empty(3, dtype=torch.float64, device=dev)
    seq = [theta, (1.2, 0.08, 0.5), (0.9, 0.12, 0.7)]
    for th in seq:
        plan.loglik(ws, dl, dz, th, tol, out=out)
    torch.cuda.synchronize()
    gc.collect()
    gc.disable()
    try:
        counts_before = B.alloc_counts()
        free_before = torch.cuda.mem_get_info(dev)[0]
        for _ in range(2):
            for th in seq:
                plan.loglik(ws, dl, dz, th, tol, out=out)
        torch.cuda.synchronize()
        free_after = torch.cuda.mem_get_info(dev)[0]
        counts_after = B.alloc_counts()
    finally:
        gc.enable()
    print(f"{precision}: pooled (pinned, streams) {counts_before} -> {counts_after}; device bytes taken "
          f"{free_before - free_after}", flush=True)
    assert counts_after == counts_before
    assert free_before - free_after <= 8 << 20


@pytest.mark.parametrize("precision", ["fp64", "mixed_fp32"])
def test_rank_budget_sizes_the_factor_arena(precision):
    """A workspace sized by the ranks a problem has (the sum of Sigma's and
    L's off-diagonal ranks) gives bitwise the result of the default
    (maxrank per tile); a budget below Sigma's rank sum stops with
    TLR_ARENA_OVERFLOW and l = -inf."""
    device()
    theta, nb, tol = (1.0, 0.1, 0.5), 200, 1e-9
    locs, z = make_problem(40, theta, "hilbert")
    dl, dz = to_dev(locs), to_dev(z)
    full = B.Plan(1600, nb, precision=precision)
    ws = full.workspace()
    ref = full.loglik(ws, dl, dz, theta, tol).cpu().numpy()
    low = np.tril_indices(full.nt, -1)
    rs, rl = full.ranks(ws)[low], full.ranks(ws, factor=True)[low]
    budget = int(rs[rs > 0].sum() + rl[rl > 0].sum())
    tight = B.Plan(1600, nb, precision=precision, rank_budget=budget)
    assert tight.ws_bytes < full.ws_bytes
    ws2 = tight.workspace()
    got = tight.loglik(ws2, dl, dz, theta, tol).cpu().numpy()
    print(f"{precision}: rank budget {budget}, workspace {tight.ws_bytes} vs {full.ws_bytes} bytes", flush=True)
    assert got.tobytes() == ref.tobytes()
    short = B.Plan(1600, nb, precision=precision, rank_budget=int(rs[rs > 0].sum()) // 2)
    ws3 = short.workspace()
    bad = short.loglik(ws3, dl, dz, theta, tol).cpu().numpy()
    assert bad[2] == -np.inf
    assert short.status(ws3)["code"] == 19
