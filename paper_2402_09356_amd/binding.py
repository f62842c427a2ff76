"""ctypes binding of include/tlrmle.h (argument marshalling only).

Tensors must be CUDA (HIP) tensors of the documented dtype and shape; the
binding passes their data pointers and the current stream to the library.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np
import torch

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtlrmle.so")

ORDERINGS = {"none": 0, "random": 1, "morton": 2, "hilbert": 3, "kdtree": 4}
PRECISIONS = {"fp64": 0, "mixed_fp32": 1}
STATUS = {0: "TLR_OK", 1: "TLR_E_INVAL", 2: "TLR_E_NOMEM", 3: "TLR_E_UNSUPPORTED", 4: "TLR_E_HIP",
          16: "TLR_NOT_SPD", 17: "TLR_RANK_OVERFLOW", 18: "TLR_E_DOMAIN", 19: "TLR_ARENA_OVERFLOW"}


class TlrError(RuntimeError):
    def __init__(self, code: int, what: str):
        super().__init__(f"{what}: {STATUS.get(code, code)}")
        self.code = code


def status_name(code: int) -> str:
    return STATUS.get(code, str(code))


class _Theta(ctypes.Structure):
    _fields_ = [("sigma2", ctypes.c_double), ("beta", ctypes.c_double), ("nu", ctypes.c_double)]


class _ThetaBiv(ctypes.Structure):
    _fields_ = [("sigma2_11", ctypes.c_double), ("sigma2_22", ctypes.c_double), ("a", ctypes.c_double),
                ("nu_11", ctypes.c_double), ("nu_22", ctypes.c_double), ("beta_12", ctypes.c_double)]


class _Tgh(ctypes.Structure):
    _fields_ = [("xi", ctypes.c_double), ("omega", ctypes.c_double), ("g", ctypes.c_double), ("h", ctypes.c_double)]


class KStat(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 48), ("launches", ctypes.c_int64), ("total_ms", ctypes.c_double),
                ("exact_launches", ctypes.c_int64), ("exact_ms", ctypes.c_double), ("flops", ctypes.c_double),
                ("bytes", ctypes.c_double)]


class DevInfo(ctypes.Structure):
    _fields_ = [("code", ctypes.c_int32), ("tile_i", ctypes.c_int32), ("tile_j", ctypes.c_int32),
                ("max_rank", ctypes.c_int32), ("rank_sum", ctypes.c_int64)]


_lib = None

P = ctypes.c_void_p
I32, I64, U32, U64, F64, SZ = (ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32, ctypes.c_uint64,
                               ctypes.c_double, ctypes.c_size_t)

_SIGNATURES = {
    "tlr_reorder_ws_bytes": (SZ, [I64, I32]),
    "tlr_reorder": (I32, [P, I64, I32, U64, U32, P, P, SZ, P]),
    "tlr_reorder_noalloc": (I32, [P, I64, I32, U64, U32, P, P]),
    "tlr_reorder_noalloc_max_n": (I64, []),
    "tlr_apply_perm": (I32, [P, I64, P, P, P, P, I32, P]),
    "tlr_plan_create": (I32, [ctypes.POINTER(P), I64, I32, I32, I32, U32]),
    "tlr_plan_destroy": (None, [P]),
    "tlr_plan_ws_bytes": (SZ, [P, I64]),
    "tlr_plan_shape": (None, [P, ctypes.POINTER(I64), ctypes.POINTER(I32), ctypes.POINTER(I32),
                              ctypes.POINTER(I32)]),
    "tlr_gen_tiles": (I32, [P, P, _Theta, P, SZ, P]),
    "tlr_compress": (I32, [P, F64, P, SZ, P, P]),
    "tlr_potrf": (I32, [P, P, SZ, P]),
    "tlr_solve_logdet": (I32, [P, P, P, SZ, P, P]),
    "tlr_loglik": (I32, [P, P, P, _Theta, F64, P, SZ, P, P, P]),
    "tlr_tgh_inverse": (I32, [P, I64, _Tgh, P, P]),
    "tlr_gen_tiles_bivariate": (I32, [P, P, _ThetaBiv, P, SZ, P]),
    "tlr_loglik_bivariate": (I32, [P, P, P, _ThetaBiv, F64, P, SZ, P, P, P]),
    "tlr_loglik_tgh": (I32, [P, P, P, _Theta, _Tgh, F64, P, SZ, P, P, P]),
    "tlr_batch_plan_create": (I32, [ctypes.POINTER(P), I32, P, P, I32, I32, U32]),
    "tlr_batch_plan_destroy": (None, [P]),
    "tlr_batch_ws_bytes": (SZ, [P]),
    "tlr_batch_status_read": (I32, [P, P, I32, ctypes.POINTER(DevInfo), P]),
    "tlr_loglik_batched": (I32, [P, P, P, P, F64, P, SZ, P, I32, P]),
    "tlr_status_read": (I32, [P, P, ctypes.POINTER(DevInfo), P]),
    "tlr_strerror": (ctypes.c_char_p, [I32]),
    "tlr_version": (ctypes.c_char_p, []),
    "tlr_diag_gemm": (I32, [I32, I32, I32, I32, I32, F64, P, I32, P, I32, F64, P, I32, P]),
    "tlr_diag_svd": (I32, [I32, I32, P, F64, P, P, P, P, P]),
    "tlr_diag_peak_hbm": (I32, [P, P, I64, I32, ctypes.POINTER(F64), P]),
    "tlr_diag_alloc_counts": (I32, [ctypes.POINTER(I64), ctypes.POINTER(I64)]),
    "tlr_diag_peak_mfma_f64": (I32, [P, I64, I32, ctypes.POINTER(F64), P]),
    "tlr_diag_gemm_strided": (I32, [I32, I32, I32, I32, I32, I32, F64, P, I32, I64, P, I32, I64, F64, P, I32, I64,
                                    P]),
    "tlr_diag_tile": (I32, [P, P, I32, I32, P, ctypes.POINTER(I32), P]),
    "tlr_diag_cholqr": (I32, [I32, I32, P, P, P, P]),
    "tlr_kstats_enable": (I32, [I32]),
    "tlr_ranks_read": (I32, [P, P, I32, P, P]),
    "tlr_kstats_reset": (I32, []),
    "tlr_kstats_select": (I32, [ctypes.c_char_p]),
    "tlr_kstats_read": (I32, [P, I32]),
    "tlr_diag_qrcp": (I32, [I32, I32, P, F64, P, P, P, P, P]),
}


def lib():
    """The loaded HIP library; raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with `python -m paper_2402_09356_amd.build`")
        handle = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(handle, name)
            fn.restype = res
            fn.argtypes = args
        _lib = handle
    return _lib


def _stream():
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("tensor must live on the GPU")
    if not t.is_contiguous():
        raise ValueError("tensor must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _check(code, what):
    if code != 0:
        raise TlrError(code, what)


def reorder(locs: torch.Tensor, kind: str, seed: int = 0) -> torch.Tensor:
    """Ordering permutation of n x 2 float64 device locations (int32, device)."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be an n x 2 float64 tensor")
    n = locs.shape[0]
    k = ORDERINGS[kind]
    L = lib()
    ws_bytes = L.tlr_reorder_ws_bytes(n, k)
    ws = torch.empty(max(ws_bytes, 1), dtype=torch.uint8, device=locs.device)
    perm = torch.empty(max(n, 1), dtype=torch.int32, device=locs.device)[:n]
    _check(L.tlr_reorder(_ptr(locs), n, k, seed & (2 ** 64 - 1), 0, _ptr(perm), _ptr(ws), ws_bytes, _stream()),
           "tlr_reorder")
    return perm


def reorder_noalloc(locs: torch.Tensor, kind: str, seed: int = 0, perm: torch.Tensor | None = None) -> torch.Tensor:
    """tlr_reorder without a workspace (the library's fixed device scratch).
    `perm` (n int32, device) may be passed in, so that the call itself makes
    no allocation on either side."""
    if locs.dtype != torch.float64 or locs.dim() != 2 or locs.shape[1] != 2:
        raise ValueError("locs must be an n x 2 float64 tensor")
    n = locs.shape[0]
    if perm is None:
        perm = torch.empty(max(n, 1), dtype=torch.int32, device=locs.device)[:n]
    _check(lib().tlr_reorder_noalloc(_ptr(locs), n, ORDERINGS[kind], seed & (2 ** 64 - 1), 0, _ptr(perm),
                                     _stream()), "tlr_reorder_noalloc")
    return perm


def tgh_inverse(t: torch.Tensor, tgh, out: torch.Tensor | None = None) -> torch.Tensor:
    """z = tau^-1((t - xi)/omega) for tgh = (xi, omega, g, h) (tlr_tgh_inverse)."""
    if t.dtype != torch.float64 or t.dim() != 1:
        raise ValueError("t must be a 1-D float64 tensor")
    out = torch.empty_like(t) if out is None else out
    _check(lib().tlr_tgh_inverse(_ptr(t), t.numel(), _Tgh(*map(float, tgh)), _ptr(out), _stream()),
           "tlr_tgh_inverse")
    return out


def apply_perm(perm: torch.Tensor, locs: torch.Tensor, z: torch.Tensor | None = None, dequantize: bool = False):
    n = locs.shape[0]
    locs_out = torch.empty_like(locs)
    z_out = torch.empty_like(z) if z is not None else None
    _check(lib().tlr_apply_perm(_ptr(perm), n, _ptr(locs), _ptr(z), _ptr(locs_out), _ptr(z_out), int(dequantize),
                                _stream()), "tlr_apply_perm")
    return locs_out, z_out


class Plan:
    """Owns a tlr_plan handle; workspaces are torch uint8 device tensors."""

    def __init__(self, n: int, nb: int, maxrank: int = 0, precision: str = "fp64", dense_tiles: bool = False,
                 truncation: str = "qrcp", rank_budget: int = 0):
        """dense_tiles: keep over-rank off-diagonal tiles dense (TLR_PLAN_DENSE_TILES);
        truncation: "qrcp" (pivoted QR, default) or "svd" (TLR_PLAN_SVD_TRUNCATION);
        rank_budget: total factor-slot width of the workspace (0: maxrank per tile)."""
        L = lib()
        h = ctypes.c_void_p()
        flags = (1 if dense_tiles else 0) | (2 if truncation == "svd" else 0)
        if truncation not in ("qrcp", "svd"):
            raise ValueError("truncation must be 'qrcp' or 'svd'")
        _check(L.tlr_plan_create(ctypes.byref(h), n, nb, maxrank, PRECISIONS[precision], flags),
               "tlr_plan_create")
        self.truncation = truncation
        self.precision = precision
        self._h = h
        self.n = n
        self.nb = nb
        n_, nb_, nt_, mr_ = I64(), I32(), I32(), I32()
        L.tlr_plan_shape(h, ctypes.byref(n_), ctypes.byref(nb_), ctypes.byref(nt_), ctypes.byref(mr_))
        self.nt = nt_.value
        self.maxrank = mr_.value
        self.rank_budget = int(rank_budget)
        self.ws_bytes = L.tlr_plan_ws_bytes(h, self.rank_budget)

    def close(self):
        if getattr(self, "_h", None):
            lib().tlr_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def gen_tiles(self, ws, locs, theta):
        _check(lib().tlr_gen_tiles(self._h, _ptr(locs), _Theta(*map(float, theta)), _ptr(ws), ws.numel(),
                                   _stream()), "tlr_gen_tiles")

    def compress(self, ws, tol, ranks: torch.Tensor | None = None):
        _check(lib().tlr_compress(self._h, float(tol), _ptr(ws), ws.numel(), _ptr(ranks), _stream()),
               "tlr_compress")

    def potrf(self, ws):
        _check(lib().tlr_potrf(self._h, _ptr(ws), ws.numel(), _stream()), "tlr_potrf")

    def solve_logdet(self, ws, z, out=None):
        out = torch.empty(3, dtype=torch.float64, device=z.device) if out is None else out
        _check(lib().tlr_solve_logdet(self._h, _ptr(z), _ptr(ws), ws.numel(), _ptr(out), _stream()),
               "tlr_solve_logdet")
        return out

    def loglik(self, ws, locs, z, theta, tol, out=None, ranks=None):
        out = torch.empty(3, dtype=torch.float64, device=z.device) if out is None else out
        _check(lib().tlr_loglik(self._h, _ptr(locs), _ptr(z), _Theta(*map(float, theta)), float(tol), _ptr(ws),
                                ws.numel(), _ptr(out), _ptr(ranks), _stream()), "tlr_loglik")
        return out

    def loglik_bivariate(self, ws, locs, z, theta, tol, out=None, ranks=None):
        """Bivariate Matern log-likelihood (tlr_loglik_bivariate): the plan's n
        is 2 x the number of locations; theta = (sigma2_11, sigma2_22, a, nu_11,
        nu_22, beta_12); z location-major (z[2p + v] = Z_v(s_p))."""
        out = torch.empty(3, dtype=torch.float64, device=z.device) if out is None else out
        _check(lib().tlr_loglik_bivariate(self._h, _ptr(locs), _ptr(z), _ThetaBiv(*map(float, theta)), float(tol),
                                          _ptr(ws), ws.numel(), _ptr(out), _ptr(ranks), _stream()),
               "tlr_loglik_bivariate")
        return out

    def loglik_tgh(self, ws, locs, t, theta, tgh, tol, z=None, out=None):
        """Tukey g-and-h log-likelihood (tlr_loglik_tgh): tgh = (xi, omega, g, h);
        out = {logdet, quad, l_TGH, sum log(omega tau'(z))}, z the transformed
        observations."""
        z = torch.empty_like(t) if z is None else z
        out = torch.empty(4, dtype=torch.float64, device=t.device) if out is None else out
        _check(lib().tlr_loglik_tgh(self._h, _ptr(locs), _ptr(t), _Theta(*map(float, theta)),
                                    _Tgh(*map(float, tgh)), float(tol), _ptr(ws), ws.numel(), _ptr(z), _ptr(out),
                                    _stream()), "tlr_loglik_tgh")
        return out

    def tile(self, ws, i, j):
        """(nb x nb numpy array of tile (i, j) in row-major math layout, rank)."""
        out = torch.empty(self.nb, self.nb, dtype=torch.float64, device=ws.device)
        r = I32()
        _check(lib().tlr_diag_tile(self._h, _ptr(ws), i, j, _ptr(out), ctypes.byref(r), _stream()),
               "tlr_diag_tile")
        return out.t().cpu().numpy(), r.value

    def ranks(self, ws, factor: bool = False) -> np.ndarray:
        """nt x nt per-tile ranks (Sigma's compressed tiles, or L's with factor)."""
        out = torch.zeros(self.nt * self.nt, dtype=torch.int32, device=ws.device)
        _check(lib().tlr_ranks_read(self._h, _ptr(ws), 1 if factor else 0, _ptr(out), _stream()), "tlr_ranks_read")
        return out.cpu().numpy().reshape(self.nt, self.nt)

    def status(self, ws) -> dict:
        info = DevInfo()
        _check(lib().tlr_status_read(self._h, _ptr(ws), ctypes.byref(info), _stream()), "tlr_status_read")
        return {"code": info.code, "name": status_name(info.code), "tile": (info.tile_i, info.tile_j),
                "max_rank": info.max_rank, "rank_sum": info.rank_sum}


class BatchPlan:
    """Owns a tlr_batch_plan: one plan per problem, one workspace for all."""

    def __init__(self, ns, nbs, maxrank: int = 0, precision: str = "fp64", dense_tiles: bool = False):
        L = lib()
        count = len(ns)
        n_arr = (ctypes.c_int64 * count)(*[int(v) for v in ns])
        nb_arr = (ctypes.c_int32 * count)(*[int(v) for v in nbs])
        h = ctypes.c_void_p()
        _check(L.tlr_batch_plan_create(ctypes.byref(h), count, ctypes.cast(n_arr, P), ctypes.cast(nb_arr, P),
                                       maxrank, PRECISIONS[precision], 1 if dense_tiles else 0),
               "tlr_batch_plan_create")
        self._h = h
        self.count = count
        self.ns = list(ns)
        self.ws_bytes = L.tlr_batch_ws_bytes(h)

    def close(self):
        if getattr(self, "_h", None):
            lib().tlr_batch_plan_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def workspace(self, device="cuda") -> torch.Tensor:
        return torch.empty(self.ws_bytes, dtype=torch.uint8, device=device)

    def loglik(self, ws, locs, zs, thetas, tol, workers: int = 8, out=None):
        """locs, zs: lists of device tensors (one per problem); returns count x 3."""
        count = self.count
        if len(locs) != count or len(zs) != count or len(thetas) != count:
            raise ValueError("one location set, observation vector and theta per problem")
        for t in list(locs) + list(zs):
            _ptr(t)
        lp = (ctypes.c_void_p * count)(*[t.data_ptr() for t in locs])
        zp = (ctypes.c_void_p * count)(*[t.data_ptr() for t in zs])
        th = (_Theta * count)(*[_Theta(*map(float, t)) for t in thetas])
        out = torch.empty(count, 3, dtype=torch.float64, device=ws.device) if out is None else out
        _check(lib().tlr_loglik_batched(self._h, ctypes.cast(lp, P), ctypes.cast(zp, P), ctypes.cast(th, P),
                                        float(tol), _ptr(ws), ws.numel(), _ptr(out), int(workers), _stream()),
               "tlr_loglik_batched")
        return out

    def status(self, ws, index: int) -> dict:
        info = DevInfo()
        _check(lib().tlr_batch_status_read(self._h, _ptr(ws), int(index), ctypes.byref(info), _stream()),
               "tlr_batch_status_read")
        return {"code": info.code, "name": status_name(info.code), "tile": (info.tile_i, info.tile_j),
                "max_rank": info.max_rank, "rank_sum": info.rank_sum}


def diag_gemm(a, b, c, alpha=1.0, beta=0.0, trans_a=False, trans_b=False):
    """c = alpha op(a) op(b) + beta c with column-major views of row-major torch tensors.

    Column-major M x K data is a row-major K x M tensor; callers pass
    tensors holding the transposes (``t().contiguous()``)."""
    M = c.shape[1]
    N = c.shape[0]
    K = a.shape[0] if not trans_a else a.shape[1]
    lda, ldb, ldc = a.shape[1], b.shape[1], c.shape[1]
    _check(lib().tlr_diag_gemm(int(trans_a), int(trans_b), M, N, K, float(alpha), _ptr(a), lda, _ptr(b), ldb,
                               float(beta), _ptr(c), ldc, _stream()), "tlr_diag_gemm")
    return c


def diag_gemm_strided(a, b, c, trans_a=False, trans_b=False, alpha=1.0, beta=0.0):
    """Batched c[t] = alpha op(a[t]) op(b[t]) + beta c[t] over the leading index.

    a, b, c: count x cols x rows device tensors holding column-major matrices
    (c[t] is M x N column-major, i.e. an N x M row-major slice)."""
    count, N, M = c.shape
    K = a.shape[1] if not trans_a else a.shape[2]
    _check(lib().tlr_diag_gemm_strided(int(trans_a), int(trans_b), count, M, N, K, float(alpha), _ptr(a),
                                       a.shape[2], a.shape[1] * a.shape[2], _ptr(b), b.shape[2],
                                       b.shape[1] * b.shape[2], float(beta), _ptr(c), M, M * N, _stream()),
           "tlr_diag_gemm_strided")
    return c


def alloc_counts() -> tuple[int, int]:
    """(pinned host buffers, streams) the library has created and pooled so far."""
    a, b = I64(), I64()
    _check(lib().tlr_diag_alloc_counts(ctypes.byref(a), ctypes.byref(b)), "tlr_diag_alloc_counts")
    return a.value, b.value


def peak_hbm(gib: float = 4.0, reps: int = 10, device="cuda") -> float:
    """Measured streaming-copy bandwidth in GB/s (read + write bytes)."""
    nbytes = int(gib * 2**30) // 16 * 16
    src = torch.ones(nbytes // 8, dtype=torch.float64, device=device)
    dst = torch.empty_like(src)
    out = F64()
    _check(lib().tlr_diag_peak_hbm(_ptr(src), _ptr(dst), nbytes, reps, ctypes.byref(out), _stream()),
           "tlr_diag_peak_hbm")
    return out.value


def peak_mfma_f64(iters: int = 20000, device="cuda") -> float:
    """Measured FP64 matrix-core rate in TFLOP/s."""
    cus = torch.cuda.get_device_properties(device).multi_processor_count
    scratch = torch.empty(512 * cus, dtype=torch.float64, device=device)
    out = F64()
    _check(lib().tlr_diag_peak_mfma_f64(_ptr(scratch), scratch.numel(), iters, ctypes.byref(out), _stream()),
           "tlr_diag_peak_mfma_f64")
    return out.value


def diag_svd(mats: torch.Tensor, tol: float):
    """mats: count x k x k (each stored column-major, i.e. the tensor holds A^T)."""
    count, k, _ = mats.shape
    S = torch.empty(count, k, dtype=torch.float64, device=mats.device)
    X = torch.empty(count, k, k, dtype=torch.float64, device=mats.device)
    rank = torch.empty(count, dtype=torch.int32, device=mats.device)
    scratch = torch.empty(512 + count * (8 * k * k + 144), dtype=torch.uint8, device=mats.device)
    _check(lib().tlr_diag_svd(count, k, _ptr(mats), float(tol), _ptr(S), _ptr(X), _ptr(rank), _ptr(scratch),
                              _stream()), "tlr_diag_svd")
    return S, X, rank


def diag_cholqr(Y: torch.Tensor):
    """Y: k x m tensor holding an m x k column-major panel.  Returns (Q, R) as
    (k x m tensor of Q's column-major data, k x k tensor of R's)."""
    k, m = Y.shape
    Q = Y.clone()
    R = torch.empty(k, k, dtype=torch.float64, device=Y.device)
    scratch = torch.empty(512 + 7 * 8 * k * k + 4096, dtype=torch.uint8, device=Y.device)
    _check(lib().tlr_diag_cholqr(m, k, _ptr(Q), _ptr(R), _ptr(scratch), _stream()), "tlr_diag_cholqr")
    return Q, R


def diag_qrcp(mats: torch.Tensor, tol: float):
    """mats: count x k x k (column-major data).  Returns (X, Bt, rank)."""
    count, k, _ = mats.shape
    X = torch.zeros(count, k, k, dtype=torch.float64, device=mats.device)
    Bt = torch.zeros(count, k, k, dtype=torch.float64, device=mats.device)
    rank = torch.empty(count, dtype=torch.int32, device=mats.device)
    scratch = torch.empty(512 + count * (8 * k * k + 144), dtype=torch.uint8, device=mats.device)
    _check(lib().tlr_diag_qrcp(count, k, _ptr(mats), float(tol), _ptr(X), _ptr(Bt), _ptr(rank), _ptr(scratch),
                               _stream()), "tlr_diag_qrcp")
    return X, Bt, rank


def kstats_enable(on: bool = True):
    """Time every instrumented launch with HIP events on its stream."""
    _check(lib().tlr_kstats_enable(1 if on else 0), "tlr_kstats_enable")


def kstats_select(name: str | None = None):
    """Time only kernel class `name` (None: every class)."""
    _check(lib().tlr_kstats_select(name.encode() if name else None), "tlr_kstats_select")


def kstats_reset():
    _check(lib().tlr_kstats_reset(), "tlr_kstats_reset")


def kstats() -> list[dict]:
    """Per-kernel launch statistics, largest total time first."""
    n = lib().tlr_kstats_read(None, 0)
    arr = (KStat * max(n, 1))()
    n = lib().tlr_kstats_read(ctypes.cast(arr, ctypes.c_void_p), n)
    out = []
    for k in arr[:n]:
        out.append({"name": k.name.decode(), "launches": k.launches, "total_ms": k.total_ms,
                    "exact_launches": k.exact_launches, "exact_ms": k.exact_ms, "flops": k.flops,
                    "bytes": k.bytes})
    return sorted(out, key=lambda d: -d["total_ms"])
