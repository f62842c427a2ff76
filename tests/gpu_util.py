"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest
import torch


def device():
    if not torch.cuda.is_available():
        pytest.fail("GPU test collected but no GPU is visible")
    return torch.device("cuda:0")


def to_dev(a, dtype=torch.float64):
    return torch.from_numpy(np.ascontiguousarray(a)).to(device=device(), dtype=dtype)


def colmajor(a):
    """Device tensor whose memory is the column-major layout of matrix a."""
    return to_dev(np.ascontiguousarray(np.asarray(a).T))


def from_colmajor(t):
    return t.cpu().numpy().T
