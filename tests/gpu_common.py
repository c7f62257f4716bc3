"""Helpers shared by the GPU parity tests (no clustering arithmetic here)."""

import sys

import numpy as np
import pytest


def say(*a):
    print("[case]", *a, flush=True)
    sys.stdout.flush()


def require_gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("GPU tests need a ROCm GPU (torch.cuda.is_available() is False)")
    from paper_2403_18766_amd import _lib
    _lib.load()  # raises if the library was not built
    return torch.device("cuda:0")


def to_dev(a, dev):
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).to(dev)


def ulp_diff_f32(a, b):
    """Elementwise distance in units in the last place between float32 arrays."""
    a = np.asarray(a, np.float32).view(np.int32).astype(np.int64)
    b = np.asarray(b, np.float32).view(np.int32).astype(np.int64)
    a = np.where(a < 0, -(a & 0x7FFFFFFF), a)
    b = np.where(b < 0, -(b & 0x7FFFFFFF), b)
    return np.abs(a - b)
