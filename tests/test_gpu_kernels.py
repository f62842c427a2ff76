"""Building blocks through the C ABI: the float64 matrix-core GEMM and the
one-sided Jacobi SVD, against NumPy."""
import numpy as np
import scipy.linalg
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


@pytest.mark.parametrize("k", [16, 64, 112, 124, 125, 150, 176, 200])
def test_cholqr_rank_deficient_panel(k):
    """The four-pass CholeskyQR: Q orthonormal on its live columns, Y = Q R,
    singular values of R equal those of Y down to rounding."""
    device()
    m = 900
    rng = np.random.default_rng(k)
    r = max(1, k // 2)
    Y = rng.standard_normal((m, r)) @ (rng.standard_normal((r, k)) * np.logspace(0, -11, r)[:, None])
    Y += 1e-17 * rng.standard_normal((m, k))
    Qt, Rt = B.diag_cholqr(colmajor(Y))
    torch.cuda.synchronize()
    Q, R = from_colmajor(Qt), from_colmajor(Rt)
    np.testing.assert_allclose(Q @ R, Y, rtol=0, atol=1e-14 * np.linalg.norm(Y, 2))
    live = np.linalg.norm(Q, axis=0) > 0.5
    G = Q[:, live].T @ Q[:, live]
    assert np.max(np.abs(G - np.eye(live.sum()))) < 1e-13
    sy = np.linalg.svd(Y, compute_uv=False)
    sr = np.linalg.svd(R, compute_uv=False)
    np.testing.assert_allclose(sr, sy, rtol=0, atol=1e-13 * sy[0])


@pytest.mark.parametrize("k", [16, 64, 65, 112, 113, 150, 176, 192, 193, 240])
def test_qrcp_truncation(k):
    """Truncated pivoted QR: ||A - Q1 B||_2 <= tol, Q1 orthonormal, rank at
    least the singular-value rank and equal (up to a pivot tie) to the first
    step at which LAPACK's pivoted QR has trailing Frobenius norm <= tol."""
    device()
    rng = np.random.default_rng(100 + k)
    mats = []
    for t in range(3):
        u, _ = np.linalg.qr(rng.standard_normal((k, k)))
        v, _ = np.linalg.qr(rng.standard_normal((k, k)))
        s = 10.0 * np.exp(-np.arange(k) * (25.0 / k))
        mats.append((u * s) @ v.T)
    tol = 1e-7
    X, Bt, rank = B.diag_qrcp(torch.stack([colmajor(a) for a in mats]), tol)
    torch.cuda.synchronize()
    X, Bt, rank = X.cpu().numpy(), Bt.cpu().numpy(), rank.cpu().numpy()
    for t in range(3):
        r = int(rank[t])
        Q1 = X[t].T[:, :r]
        Bm = Bt[t].T[:, :r].T
        err = np.linalg.norm(mats[t] - Q1 @ Bm, 2)
        assert err <= tol * 1.0001, (k, t, r, err)
        assert np.max(np.abs(Q1.T @ Q1 - np.eye(r))) < 1e-13
        svr = int(np.count_nonzero(np.linalg.svd(mats[t], compute_uv=False) > tol))
        Rl = scipy.linalg.qr(mats[t], pivoting=True, mode="r")[0]
        rl = next(c for c in range(k + 1) if np.linalg.norm(Rl[c:, c:]) <= tol)
        assert svr <= r and abs(r - rl) <= 1, (r, rl, svr)
