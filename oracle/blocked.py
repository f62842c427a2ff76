"""Blocked dense Cholesky likelihood for problems whose covariance does not
fit in memory as one array (paper Section 1, eq. "loglik"; Section 5.3.1 runs
up to n = 90,000).

TEST INFRASTRUCTURE ONLY (see the package docstring).

This is the dense oracle of ``likelihood`` cut into b x b blocks, nothing
more: Sigma(theta) is never compressed.  Only the blocks on and below the
diagonal are formed (Sigma is symmetric), each from the covariance function of
``matern``.  The factor is the textbook right-looking blocked Cholesky
factorisation, with the same arithmetic as the unblocked one up to the order
of the sums:

    for k = 0 .. nb-1:
        L_kk = chol(A_kk)                      (LAPACK, lower)
        L_ik = A_ik L_kk^-T            i > k   (triangular solve)
        A_ij = A_ij - L_ik L_jk^T      i >= j > k

and then log|Sigma| = 2 sum log diag(L_kk), y = L^-1 Z by blocked forward
substitution, quad = y^T y.  A Cholesky failure of a diagonal block means
Sigma is not positive definite.

Blocks live in a dict of arrays, or -- for n = 90,000, whose lower triangle
alone is 32 GB -- in one memory-mapped file of b x b slots, so that the page
cache rather than the process holds them.
"""
from __future__ import annotations

import os

import numpy as np
from scipy import linalg

from . import likelihood, matern


def block_bounds(n: int, b: int):
    nblk = (n + b - 1) // b
    return [(k * b, min((k + 1) * b, n)) for k in range(nblk)]


class _Store:
    """Lower-triangular block storage: in memory, or one memory-mapped file."""

    def __init__(self, n: int, b: int, path: str | None):
        self.bounds = block_bounds(n, b)
        self.nblk = len(self.bounds)
        self.b = b
        self.path = path
        if path is None:
            self.mem = {}
            self.mm = None
        else:
            count = self.nblk * (self.nblk + 1) // 2
            self.mm = np.memmap(path, dtype=np.float64, mode="w+", shape=(count, b, b))
            self.mem = None

    def _slot(self, i: int, j: int) -> int:
        return i * (i + 1) // 2 + j

    def get(self, i: int, j: int) -> np.ndarray:
        if self.mem is not None:
            return self.mem[(i, j)]
        r = self.bounds[i][1] - self.bounds[i][0]
        c = self.bounds[j][1] - self.bounds[j][0]
        return self.mm[self._slot(i, j), :r, :c]

    def put(self, i: int, j: int, a: np.ndarray) -> None:
        if self.mem is not None:
            self.mem[(i, j)] = np.array(a, dtype=np.float64, copy=True)
        else:
            r, c = a.shape
            self.mm[self._slot(i, j), :r, :c] = a

    def close(self) -> None:
        if self.mm is not None:
            path = self.path
            del self.mm
            self.mm = None
            os.remove(path)


def _truncate_tiles(block: np.ndarray, r0: int, c0: int, nb: int, tol: float, maxrank: int) -> None:
    """Replace every strictly-lower nb x nb tile (P > Q, global tile indices)
    inside a block whose first row / column are r0 / c0 by its SVD truncated
    at tol (singular values > tol kept; a tile above maxrank stays exact) --
    the tile-truncated covariance of ``tlr.compressed_matrix``, block by block."""
    rows, cols = block.shape
    for pr in range(r0 // nb, (r0 + rows + nb - 1) // nb):
        for qc in range(c0 // nb, (c0 + cols + nb - 1) // nb):
            if pr <= qc:
                continue
            a0, a1 = max(pr * nb, r0) - r0, min((pr + 1) * nb, r0 + rows) - r0
            b0, b1 = max(qc * nb, c0) - c0, min((qc + 1) * nb, c0 + cols) - c0
            u, sv, vt = np.linalg.svd(block[a0:a1, b0:b1], full_matrices=False)
            r = int(np.count_nonzero(sv > tol))
            if r <= maxrank:
                block[a0:a1, b0:b1] = (u[:, :r] * sv[:r]) @ vt[:r, :]


class BlockedCholesky:
    """Lower Cholesky factor of Sigma(theta) held as b x b blocks.

    With ``tiles = (nb, tol, maxrank)`` the factor is that of the
    tile-truncated covariance instead (paper Section 2: every off-diagonal
    nb x nb tile replaced by its truncated SVD), for the error that
    compression alone causes; b must then be a multiple of nb."""

    def __init__(self, locs: np.ndarray, theta, b: int = 4096, path: str | None = None, log=None, tiles=None):
        locs = np.asarray(locs, dtype=np.float64)
        self.n = locs.shape[0]
        self.store = _Store(self.n, b, path)
        bd = self.store.bounds
        nblk = self.store.nblk
        if tiles is not None and b % tiles[0] != 0:
            raise ValueError("the block size must be a multiple of the tile size")
        # Sigma's blocks on and below the diagonal
        for i in range(nblk):
            for j in range(i + 1):
                blk = matern.covariance(locs[bd[i][0]:bd[i][1]], locs[bd[j][0]:bd[j][1]], theta)
                if tiles is not None:
                    _truncate_tiles(blk, bd[i][0], bd[j][0], *tiles)
                self.store.put(i, j, blk)
            if log is not None and tiles is not None:
                log(f"block row {i + 1}/{nblk} assembled")
        # right-looking blocked factorisation
        for k in range(nblk):
            try:
                lkk = linalg.cholesky(self.store.get(k, k), lower=True, check_finite=True)
            except linalg.LinAlgError as exc:
                self.close()
                raise likelihood.NotPositiveDefinite(f"block {k}: {exc}") from exc
            if np.any(np.diag(lkk) <= 0) or not np.all(np.isfinite(np.diag(lkk))):
                self.close()
                raise likelihood.NotPositiveDefinite(f"block {k}: non-positive pivot")
            self.store.put(k, k, lkk)
            for i in range(k + 1, nblk):
                # L_ik = A_ik L_kk^-T, i.e. L_kk L_ik^T = A_ik^T
                lik = linalg.solve_triangular(lkk, self.store.get(i, k).T, lower=True).T
                self.store.put(i, k, lik)
            for j in range(k + 1, nblk):
                ljk = np.array(self.store.get(j, k))
                for i in range(j, nblk):
                    self.store.put(i, j, self.store.get(i, j) - np.array(self.store.get(i, k)) @ ljk.T)
            if log is not None:
                log(f"block column {k + 1}/{nblk} factored")

    def logdet(self) -> float:
        """log|Sigma| = 2 sum_k sum log diag(L_kk)."""
        return 2.0 * float(sum(np.sum(np.log(np.diag(self.store.get(k, k)))) for k in range(self.store.nblk)))

    def solve(self, z: np.ndarray) -> np.ndarray:
        """y = L^-1 z by blocked forward substitution."""
        z = np.asarray(z, dtype=np.float64)
        bd = self.store.bounds
        y = np.zeros(self.n)
        for i in range(self.store.nblk):
            r0, r1 = bd[i]
            rhs = z[r0:r1].copy()
            for k in range(i):
                rhs -= np.array(self.store.get(i, k)) @ y[bd[k][0]:bd[k][1]]
            y[r0:r1] = linalg.solve_triangular(self.store.get(i, i), rhs, lower=True)
        return y

    def matvec(self, e: np.ndarray) -> np.ndarray:
        """L e (used to draw Z ~ N(0, Sigma) from white noise e)."""
        e = np.asarray(e, dtype=np.float64)
        bd = self.store.bounds
        out = np.zeros(self.n)
        for i in range(self.store.nblk):
            r0, r1 = bd[i]
            acc = np.tril(self.store.get(i, i)) @ e[r0:r1]
            for k in range(i):
                acc = acc + np.array(self.store.get(i, k)) @ e[bd[k][0]:bd[k][1]]
            out[r0:r1] = acc
        return out

    def loglik(self, z: np.ndarray) -> likelihood.LogLik:
        """eq. "loglik" from this factor: -(n/2) log 2 pi - logdet/2 - y^T y / 2."""
        y = self.solve(z)
        logdet = self.logdet()
        quad = float(y @ y)
        ll = -0.5 * self.n * likelihood.LOG_2PI - 0.5 * logdet - 0.5 * quad
        return likelihood.LogLik(ll, logdet, quad, self.n)

    def close(self) -> None:
        self.store.close()


def loglik_blocked(locs, z, theta, b: int = 4096, path: str | None = None, log=None,
                   tiles=None) -> likelihood.LogLik:
    """l(theta) by the blocked factorisation (raises NotPositiveDefinite);
    tiles = (nb, tol, maxrank) gives l of the tile-truncated covariance."""
    f = BlockedCholesky(locs, theta, b, path, log, tiles)
    try:
        return f.loglik(z)
    finally:
        f.close()
