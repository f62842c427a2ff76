"""Pins of the oracle's tile ranks and tile-truncated likelihood
(paper Sections 2-3 and Table 'memory' of Section 5.2)."""
import json
import os

import numpy as np
import pytest

import synthetic
from oracle import likelihood as L
from oracle import matern as M
from oracle import ordering as O
from oracle import tlr as T


def _setup(m=20, seed=3, theta=(1.0, 0.1, 0.5), kind="morton"):
    locs = synthetic.jittered_grid(m, seed)
    perm = O.reorder(locs, kind)
    locs = locs[perm]
    z = L.sample_field(synthetic.jittered_grid(m, seed), theta, synthetic.standard_normal(m * m, seed + 1))[perm]
    return locs, z


def test_eckart_young_truncation_error():
    locs, _ = _setup()
    sig = M.covariance_matrix(locs, (1.0, 0.1, 0.5))
    nb, tol = 100, 1e-7
    tilde, ranks = T.compressed_matrix(sig, nb, tol)
    b = T.tile_bounds(400, nb)
    for i in range(len(b)):
        for j in range(i):
            blk = sig[b[i][0]:b[i][1], b[j][0]:b[j][1]]
            err = np.linalg.norm(blk - tilde[b[i][0]:b[i][1], b[j][0]:b[j][1]], 2)
            s = np.linalg.svd(blk, compute_uv=False)
            r = ranks[i, j]
            assert r >= 0
            nxt = s[r] if r < s.size else 0.0
            assert err == pytest.approx(nxt, rel=1e-6, abs=1e-14)
            assert nxt <= tol
    assert np.array_equal(tilde, tilde.T)


def test_tol_zero_keeps_exact_matrix_and_dense_fallback():
    locs, z = _setup(m=12)
    theta = (1.0, 0.1, 0.5)
    sig = M.covariance_matrix(locs, theta)
    tilde, ranks = T.compressed_matrix(sig, 36, 0.0)
    assert np.all(ranks[np.tril_indices(4, -1)] == T.DENSE)  # full rank > nb/2
    assert np.array_equal(tilde, sig)


def test_compressed_loglik_converges_as_tol_to_zero():
    locs, z = _setup(m=24)
    theta = (1.0, 0.1, 0.5)
    dense = L.loglik_dense(locs, z, theta).loglik
    errs = []
    for tol in (1e-3, 1e-5, 1e-7, 1e-9, 1e-12):
        ll, _ = T.compressed_loglik(locs, z, theta, 96, tol)
        errs.append(abs(ll.loglik - dense))
    assert errs[-1] < 1e-8 * 576
    assert errs[0] > errs[2] > errs[4]


def test_rank_monotone_in_tol_and_storage_accounting():
    locs, _ = _setup(m=20)
    sig = M.covariance_matrix(locs, (1.0, 0.03, 0.5))
    ts = T.tile_svd(sig, 100)
    r7, _ = T.tile_ranks(ts, 1e-7)
    r9, _ = T.tile_ranks(ts, 1e-9)
    assert np.all(r9[r7 >= 0] >= r7[r7 >= 0])
    # the dense storage of the Table 'memory' dense row: nt(nt-1)/2 * nb^2 * 8 bytes
    allden = np.full_like(r7, T.DENSE)
    assert T.storage_bytes(allden, 100, 400) == 6 * 100 * 100 * 8


@pytest.mark.parametrize("n,dense_mb", [(10000, 360), (20000, 1520), (30000, 3480), (40000, 6240)])
def test_table_memory_dense_row(golden_dir, n, dense_mb):
    tab = json.load(open(os.path.join(golden_dir, "table_memory.json")))
    assert tab["rows"][str(n)]["dense"] == dense_mb
    nt = n // 1000
    ranks = np.full((nt, nt), T.DENSE)
    assert T.storage_bytes(ranks, 1000, n) == dense_mb * 10 ** 6


def test_ordering_reduces_storage_against_random():
    locs = synthetic.uniform_points(2500, 17)
    theta = (1.0, 0.1, 0.5)
    out = {}
    for kind in ("random", "hilbert", "morton", "kdtree"):
        p = O.reorder(locs, kind, seed=3)
        sig = M.covariance_matrix(locs[p], theta)
        ranks, _ = T.tile_ranks(T.tile_svd(sig, 250), 1e-7)
        out[kind] = T.storage_bytes(ranks, 250, 2500)
    for kind in ("hilbert", "morton", "kdtree"):
        assert out[kind] < 0.5 * out["random"]


@pytest.mark.slow
def test_table_memory_magnitude_hilbert_medium(golden_dir):
    """n = 10,000, nb = 1,000, Hilbert, beta = 0.1, tol = 1e-7: storage within
    +-25% of the paper's 42 MB (one dataset instead of the paper's 100)."""
    tab = json.load(open(os.path.join(golden_dir, "table_memory.json")))
    paper_mb = tab["rows"]["10000"]["hilbert"][1]
    locs = synthetic.uniform_points(10000, 1234)
    p = O.reorder(locs, "hilbert")
    sig = M.covariance_matrix(locs[p], (1.0, 0.1, 0.5))
    ranks, _ = T.tile_ranks(T.tile_svd(sig, 1000), 1e-7)
    mb = T.storage_bytes(ranks, 1000, 10000) / 1e6
    assert 0.75 * paper_mb <= mb <= 1.25 * paper_mb, mb


def test_rank_stats_histogram():
    ranks = np.array([[0, 0, 0], [3, 0, 0], [T.DENSE, 12, 0]])
    numerical = np.array([[0, 0, 0], [3, 0, 0], [400, 12, 0]])
    st = T.rank_stats(ranks, numerical)
    assert st["dense"] == 1
    assert sum(st["hist"]) == 2
    assert st["summary"]["max"] == 400
