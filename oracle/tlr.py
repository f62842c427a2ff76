"""Exact tile ranks and the tile-truncated covariance (paper Sections 2 and 3).

The matrix is cut into nb x nb tiles; tile (i, j) covers the ordered points
[i*nb, (i+1)*nb) x [j*nb, (j+1)*nb) (the last tile row/column is shorter when
nb does not divide n).  Diagonal tiles stay dense.  Each off-diagonal tile of
the lower triangle is compressed by its SVD, keeping the singular values above
the accuracy threshold; their count is the tile rank (Section 3, opening
paragraphs; Fig. "tlr").

Readings taken here:

* The threshold is absolute: rank = #{k : s_k > tol} (strict).
* A tile whose rank exceeds maxrank (default nb/2, the storage break-even of
  Section 3) is kept dense; its numerical rank is still reported.
* The ranks histogrammed are those of Sigma's own off-diagonal tiles (lower
  triangle), before any factorisation.

The compressed-input likelihood l(Sigma~) uses Sigma~ = the matrix with every
low-rank tile replaced by its truncated SVD, and is computed densely; the
difference l(Sigma~) - l(Sigma) is the error due to compression alone.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np

from . import likelihood, matern

DENSE = -1


def tile_bounds(n: int, nb: int):
    nt = (n + nb - 1) // nb
    return [(t * nb, min((t + 1) * nb, n)) for t in range(nt)]


def default_maxrank(nb: int) -> int:
    return nb // 2


@dataclass
class TileSVD:
    n: int
    nb: int
    svals: dict = field(default_factory=dict)  # (i, j) -> singular values, i > j


def tile_svd(sigma: np.ndarray, nb: int, tiles=None) -> TileSVD:
    """Singular values of every (or the listed) lower off-diagonal tile."""
    n = sigma.shape[0]
    b = tile_bounds(n, nb)
    nt = len(b)
    out = TileSVD(n, nb)
    todo = tiles if tiles is not None else [(i, j) for i in range(nt) for j in range(i)]
    for (i, j) in todo:
        r0, r1 = b[i]
        c0, c1 = b[j]
        out.svals[(i, j)] = np.linalg.svd(sigma[r0:r1, c0:c1], compute_uv=False)
    return out


def tile_svd_from_locations(locs: np.ndarray, theta, nb: int, tiles) -> TileSVD:
    """Singular values of selected tiles, generating only those tiles."""
    n = locs.shape[0]
    b = tile_bounds(n, nb)
    out = TileSVD(n, nb)
    for (i, j) in tiles:
        r0, r1 = b[i]
        c0, c1 = b[j]
        block = matern.covariance(locs[r0:r1], locs[c0:c1], theta)
        out.svals[(i, j)] = np.linalg.svd(block, compute_uv=False)
    return out


def numerical_rank(svals: np.ndarray, tol: float) -> int:
    return int(np.count_nonzero(np.asarray(svals) > tol))


def tile_ranks(tsvd: TileSVD, tol: float, maxrank: int | None = None):
    """(ranks, numerical) nt x nt int arrays; ranks has DENSE where r > maxrank.

    Entries outside the strict lower triangle are 0.
    """
    nt = (tsvd.n + tsvd.nb - 1) // tsvd.nb
    maxrank = default_maxrank(tsvd.nb) if maxrank is None else maxrank
    ranks = np.zeros((nt, nt), dtype=np.int64)
    numerical = np.zeros((nt, nt), dtype=np.int64)
    for (i, j), s in tsvd.svals.items():
        r = numerical_rank(s, tol)
        numerical[i, j] = r
        ranks[i, j] = DENSE if r > maxrank else r
    return ranks, numerical


def rank_stats(ranks: np.ndarray, numerical: np.ndarray, bins=(0, 1, 11, 26, 51, 101, 201, 10**9)):
    """Histogram (low-rank tiles by rank bin, plus dense count) and summary."""
    nt = ranks.shape[0]
    low = [int(ranks[i, j]) for i in range(nt) for j in range(i) if ranks[i, j] != DENSE]
    dense = sum(1 for i in range(nt) for j in range(i) if ranks[i, j] == DENSE)
    hist = np.histogram(low, bins=np.asarray(bins))[0].tolist() if low else [0] * (len(bins) - 1)
    allr = [int(numerical[i, j]) for i in range(nt) for j in range(i)]
    summary = {}
    if allr:
        summary = {"min": int(np.min(allr)), "median": float(np.median(allr)),
                   "mean": float(np.mean(allr)), "max": int(np.max(allr))}
    return {"bins": list(bins), "hist": hist, "dense": int(dense), "summary": summary}


def storage_bytes(ranks: np.ndarray, nb: int, n: int, word: int = 8) -> int:
    """Bytes to hold the off-diagonal tiles: 2*rows*r words per low-rank tile
    (U and V), the full tile for dense ones."""
    b = tile_bounds(n, nb)
    nt = len(b)
    total = 0
    for i in range(nt):
        for j in range(i):
            rows = b[i][1] - b[i][0]
            cols = b[j][1] - b[j][0]
            r = int(ranks[i, j])
            total += rows * cols * word if r == DENSE else (rows + cols) * r * word
    return total


def compressed_matrix(sigma: np.ndarray, nb: int, tol: float, maxrank: int | None = None):
    """Sigma~: lower off-diagonal tiles replaced by truncated SVDs, mirrored."""
    n = sigma.shape[0]
    maxrank = default_maxrank(nb) if maxrank is None else maxrank
    b = tile_bounds(n, nb)
    out = np.array(sigma, dtype=np.float64, copy=True)
    ranks = np.zeros((len(b), len(b)), dtype=np.int64)
    for i in range(len(b)):
        for j in range(i):
            r0, r1 = b[i]
            c0, c1 = b[j]
            u, s, vt = np.linalg.svd(sigma[r0:r1, c0:c1], full_matrices=False)
            r = numerical_rank(s, tol)
            if r > maxrank:
                ranks[i, j] = DENSE
                continue
            ranks[i, j] = r
            approx = (u[:, :r] * s[:r]) @ vt[:r, :]
            out[r0:r1, c0:c1] = approx
            out[c0:c1, r0:r1] = approx.T
    return out, ranks


def compressed_loglik(locs, z, theta, nb: int, tol: float, maxrank: int | None = None):
    """(l(Sigma~), ranks); raises NotPositiveDefinite when Sigma~ is not SPD."""
    sigma = matern.covariance_matrix(locs, theta)
    tilde, ranks = compressed_matrix(sigma, nb, tol, maxrank)
    return likelihood.loglik_from_matrix(tilde, z), ranks
