"""Orderings on the GPU are bit-identical to the oracle (paper Section 3)."""
import numpy as np
import pytest
import torch

import synthetic
from oracle import ordering as O
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu

KINDS = ["none", "random", "morton", "hilbert", "kdtree"]


def _gpu_perm(locs, kind, seed=0):
    perm = B.reorder(to_dev(locs), kind, seed)
    torch.cuda.synchronize()
    return perm.cpu().numpy().astype(np.int64)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("n", [1, 2, 3, 7, 1000, 1025])
def test_small_uniform(kind, n):
    device()
    locs = synthetic.uniform_points(n, 100 + n)
    print(f"order {kind} n={n}", flush=True)
    assert np.array_equal(_gpu_perm(locs, kind, seed=42), O.reorder(locs, kind, seed=42))


@pytest.mark.parametrize("kind", KINDS)
def test_forced_ties_and_duplicates(kind):
    device()
    base = synthetic.uniform_points(300, 5)
    locs = np.concatenate([base, base[:50], base[:50] + 1e-9, np.full((20, 2), 0.5)])
    locs = np.clip(locs, 0, 1)
    print(f"order ties {kind}", flush=True)
    assert np.array_equal(_gpu_perm(locs, kind, seed=9), O.reorder(locs, kind, seed=9))


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("m", [40, 200, 300])
def test_jittered_grids_of_the_workloads(kind, m):
    """1,600 (40x40), 40,000 (200x200) and 90,000 (300x300) points."""
    device()
    locs = synthetic.jittered_grid(m, synthetic.seed_for({40: 1, 200: 2, 300: 3}[m], synthetic.SEED_LOCS))
    seed = synthetic.seed_for({40: 1, 200: 2, 300: 3}[m], synthetic.SEED_ORDER)
    print(f"order grid {kind} m={m}", flush=True)
    assert np.array_equal(_gpu_perm(locs, kind, seed), O.reorder(locs, kind, seed))


def test_domain_rejected():
    device()
    with pytest.raises(B.TlrError):
        B.reorder(to_dev(np.array([[0.2, 0.3], [1.5, 0.2]])), "morton")
    with pytest.raises(B.TlrError):
        B.reorder(to_dev(np.array([[0.2, np.nan], [0.5, 0.2]])), "hilbert")


def test_apply_perm_and_dequantize():
    device()
    locs = synthetic.uniform_points(500, 3)
    z = np.arange(500, dtype=np.float64)
    perm = O.reorder(locs, "hilbert")
    dperm = to_dev(perm, torch.int32)
    lo, zo = B.apply_perm(dperm, to_dev(locs), to_dev(z))
    torch.cuda.synchronize()
    assert np.array_equal(lo.cpu().numpy(), locs[perm])
    assert np.array_equal(zo.cpu().numpy(), z[perm])
    lq, _ = B.apply_perm(dperm, to_dev(locs), None, dequantize=True)
    torch.cuda.synchronize()
    assert np.array_equal(lq.cpu().numpy(), O.ordered_locations(locs, perm, "hilbert", dequantize_codes=True))
