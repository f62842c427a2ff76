"""The allocation-free ordering entry point against the workspace one.

tlr_reorder_noalloc runs the ordering in the library's fixed device scratch
array instead of a caller workspace.  Its permutation must equal
tlr_reorder's bit for bit, on two calls in a row with the second one smaller
(the scratch keeps the first call's contents), for every ordering kind; a size
above the stated maximum is refused before anything is enqueued; and with the
output preallocated the call changes neither torch's allocations nor the
device's free memory.
"""
import gc

import numpy as np
import pytest
import torch

import synthetic
from paper_2402_09356_amd import binding as B
from tests.gpu_util import device, to_dev

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("kind", ["none", "random", "morton", "hilbert", "kdtree"])
def test_noalloc_equals_workspace_ordering(kind):
    dev = device()
    big = to_dev(synthetic.jittered_grid(300, synthetic.seed_for(3, synthetic.SEED_LOCS)))   # n = 90,000
    small = to_dev(synthetic.uniform_points(1600, 4321))
    seed = synthetic.seed_for(3, synthetic.SEED_ORDER)
    for locs in (big, small):
        n = locs.shape[0]
        print(f"noalloc {kind} n={n}", flush=True)
        ref = B.reorder(locs, kind, seed).cpu().numpy()
        perm = torch.empty(n, dtype=torch.int32, device=dev)
        gc.collect()
        gc.disable()  # no collector run (and tensor free) inside the measured window
        try:
            torch.cuda.synchronize()
            used = torch.cuda.memory_allocated(dev)
            free_before = torch.cuda.mem_get_info(dev)[0]
            got = B.reorder_noalloc(locs, kind, seed, perm=perm)
            torch.cuda.synchronize()
            used_after = torch.cuda.memory_allocated(dev)
            free_after = torch.cuda.mem_get_info(dev)[0]
        finally:
            gc.enable()
        # nothing grows (torch may release a cached temporary meanwhile)
        assert used_after <= used
        assert free_after >= free_before
        assert np.array_equal(got.cpu().numpy(), ref)


def test_noalloc_refuses_sizes_above_its_maximum():
    dev = device()
    cap = B.lib().tlr_reorder_noalloc_max_n()
    assert cap == 131072
    locs = torch.full((cap + 1, 2), 0.5, dtype=torch.float64, device=dev)
    with pytest.raises(B.TlrError) as e:
        B.reorder_noalloc(locs, "hilbert")
    assert e.value.code == 2
    # the largest size accepted works
    ok = to_dev(synthetic.uniform_points(cap, 99))
    ref = B.reorder(ok, "morton").cpu().numpy()
    assert np.array_equal(B.reorder_noalloc(ok, "morton").cpu().numpy(), ref)
