"""Building blocks through the C ABI: the float64 matrix-core GEMM and the
one-sided Jacobi SVD, against NumPy."""
import numpy as np
import pytest
import torch

from paper_2402_09356_amd import binding as B
from tests.gpu_util import colmajor, device, from_colmajor

pytestmark = pytest.mark.gpu

SHAPES = [(1, 1, 1), (64, 64, 16), (100, 37, 203), (900, 40, 900), (130, 130, 0), (17, 250, 65), (900, 900, 7)]


@pytest.mark.parametrize("ta", [False, True])
@pytest.mark.parametrize("tb", [False, True])
@pytest.mark.parametrize("shape", SHAPES)
def test_gemm_matches_numpy(ta, tb, shape):
    device()
    M, N, K = shape
    rng = np.random.default_rng(M * 131 + N * 7 + K)
    A = rng.standard_normal((K, M) if ta else (M, K))
    Bm = rng.standard_normal((N, K) if tb else (K, N))
    C0 = rng.standard_normal((M, N))
    a, b, c = colmajor(A), colmajor(Bm), colmajor(C0)
    print(f"gemm ta={ta} tb={tb} M={M} N={N} K={K}", flush=True)
    B.diag_gemm(a, b, c, alpha=-0.75, beta=0.5, trans_a=ta, trans_b=tb)
    torch.cuda.synchronize()
    ref = -0.75 * ((A.T if ta else A) @ (Bm.T if tb else Bm)) + 0.5 * C0
    got = from_colmajor(c)
    scale = max(1.0, np.sqrt(K))
    np.testing.assert_allclose(got, ref, rtol=0, atol=1e-13 * scale)


def test_gemm_beta_zero_ignores_nan():
    device()
    rng = np.random.default_rng(1)
    A, Bm = rng.standard_normal((70, 33)), rng.standard_normal((33, 90))
    c = colmajor(np.full((70, 90), np.nan))
    B.diag_gemm(colmajor(A), colmajor(Bm), c, alpha=1.0, beta=0.0)
    torch.cuda.synchronize()
    np.testing.assert_allclose(from_colmajor(c), A @ Bm, rtol=0, atol=1e-12)


@pytest.mark.parametrize("k", [8, 40, 124, 125, 200])
def test_jacobi_svd_graded_spectrum(k):
    device()
    rng = np.random.default_rng(k)
    mats, svals = [], []
    for t in range(3):
        u, _ = np.linalg.qr(rng.standard_normal((k, k)))
        v, _ = np.linalg.qr(rng.standard_normal((k, k)))
        s = np.logspace(1, -13, k)
        mats.append((u * s) @ v.T)
        svals.append(s)
    dev = torch.stack([colmajor(a) for a in mats])
    print(f"svd k={k}", flush=True)
    S, X, rank = B.diag_svd(dev, 1e-7)
    torch.cuda.synchronize()
    S, X, rank = S.cpu().numpy(), X.cpu().numpy(), rank.cpu().numpy()
    for t in range(3):
        ref = np.linalg.svd(mats[t], compute_uv=False)
        np.testing.assert_allclose(S[t], ref, rtol=0, atol=1e-13 * ref[0])
        assert rank[t] == np.count_nonzero(ref > 1e-7)
        Xt = X[t].T  # column-major -> math
        r = int(rank[t])
        G = Xt[:, :r].T @ Xt[:, :r]
        assert np.max(np.abs(G - np.eye(r))) < 1e-10
        proj = Xt[:, :r].T @ mats[t]
        np.testing.assert_allclose(np.linalg.norm(proj, axis=1), S[t][:r], rtol=0, atol=1e-13 * ref[0])
