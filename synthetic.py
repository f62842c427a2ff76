"""Seeded synthetic inputs shared by the CPU oracle and the GPU path.

This module holds no arithmetic of the likelihood method itself: it draws
locations, standard-normal vectors, parameter perturbations, problem sizes and
arrival times from fixed seeds, and nothing else.  Observation vectors Z that
must follow N(0, Sigma(theta)) are formed by whoever owns a covariance
factorisation (the oracle in tests); this module only supplies the white noise
e with Z = L e.

Workload recipe (the paper's synthetic data live on the unit square, Section 5,
with perfect-square n in Section 5.3.1):

* jittered grid: m x m cells, point (i, j) at ((i + 1/2 + u)/m, (j + 1/2 + v)/m)
  with u, v ~ U(-0.4, 0.4), generation index i*m + j;
* i.i.d. uniform points in [0, 1]^2 for the batching workload;
* numpy Generator(PCG64(seed)) for every draw.
"""
from __future__ import annotations

import numpy as np

# Seed convention: base 1000*c for workload number c, plus a stream offset.
SEED_LOCS, SEED_Z, SEED_ORDER, SEED_SKETCH, SEED_ARRIVALS, SEED_THETA = 1, 2, 3, 4, 5, 6


def seed_for(config: int, stream: int, extra: int = 0) -> int:
    """Seed of one random stream of one workload."""
    return 1000 * int(config) + int(stream) + 10 * int(extra)


def _rng(seed: int) -> np.random.Generator:
    return np.random.Generator(np.random.PCG64(int(seed)))


def jittered_grid(m: int, seed: int, jitter: float = 0.4) -> np.ndarray:
    """m*m locations, n x 2 float64, row-major generation order (i major)."""
    rng = _rng(seed)
    u = rng.uniform(-jitter, jitter, size=(m, m))
    v = rng.uniform(-jitter, jitter, size=(m, m))
    i, j = np.meshgrid(np.arange(m), np.arange(m), indexing="ij")
    x = (i + 0.5 + u) / m
    y = (j + 0.5 + v) / m
    return np.ascontiguousarray(np.stack([x.ravel(), y.ravel()], axis=1))


def uniform_points(n: int, seed: int) -> np.ndarray:
    """n i.i.d. uniform locations in the open unit square, n x 2 float64."""
    rng = _rng(seed)
    pts = rng.uniform(0.0, 1.0, size=(n, 2))
    return np.ascontiguousarray(np.clip(pts, 1e-12, 1.0 - 1e-12))


def standard_normal(n: int, seed: int) -> np.ndarray:
    """White noise e ~ N(0, I_n) in generation order."""
    return _rng(seed).standard_normal(n)


def collinear_points(n: int, seed: int, margin: float = 0.05) -> np.ndarray:
    """n distinct points on the diagonal of the unit square, sorted along it.

    Positions t are sorted uniforms in [margin, 1 - margin]; location = (t, t).
    """
    rng = _rng(seed)
    t = np.sort(rng.uniform(margin, 1.0 - margin, size=n))
    # enforce distinctness deterministically
    for k in range(1, n):
        if t[k] <= t[k - 1]:
            t[k] = np.nextafter(t[k - 1], 2.0)
    return np.ascontiguousarray(np.stack([t, t], axis=1))


def theta_perturbations(theta, count: int, seed: int, scale: float = 0.2) -> np.ndarray:
    """count parameter vectors theta * exp(scale * N(0, I_3))."""
    rng = _rng(seed)
    base = np.asarray(theta, dtype=np.float64)
    return base[None, :] * np.exp(scale * rng.standard_normal((count, base.size)))


def batch_sizes(count: int, lo: int, hi: int, seed: int) -> np.ndarray:
    """count problem sizes drawn uniformly from the integers [lo, hi]."""
    return _rng(seed).integers(lo, hi + 1, size=count)


def batch_thetas(count: int, seed: int, nus=(0.5, 1.5, 2.5), beta_lo=0.03, beta_hi=0.3) -> np.ndarray:
    """Per-problem (sigma2=1, beta ~ U(lo, hi), nu uniform over nus)."""
    rng = _rng(seed)
    beta = rng.uniform(beta_lo, beta_hi, size=count)
    nu = np.asarray(nus, dtype=np.float64)[rng.integers(0, len(nus), size=count)]
    return np.stack([np.ones(count), beta, nu], axis=1)


def poisson_arrivals(count: int, rate: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson stream."""
    gaps = _rng(seed).exponential(1.0 / rate, size=count)
    return np.cumsum(gaps)


def sketch_uniforms(shape, seed: int) -> np.ndarray:
    """Uniform(0,1) draws for any randomised step that takes its randomness as input."""
    return _rng(seed).uniform(size=shape)
