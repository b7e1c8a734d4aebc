"""Helpers shared by the GPU tests (no oracle arithmetic here)."""
import sys

import numpy as np
import pytest


def say(*a):
    """Name the case on stdout before a GPU step (survives a lost box)."""
    print("[gpu-case]", *a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="session")
def dev():
    import torch
    import paper_2207_05152_amd as dl
    assert torch.cuda.is_available(), "GPU tests need a visible MI355X"
    dl.lib()
    dl.dlic_init(0)
    return torch.device("cuda:0")


def to_dev(a, dev, dtype=None):
    import torch
    t = torch.from_numpy(np.ascontiguousarray(a))
    if dtype is not None:
        t = t.to(dtype)
    return t.to(dev)


def cf_pack(c, f):
    """c | (f - 1) << 16 as int32 bits (the ABI's packed interval)."""
    return (np.asarray(c, np.int64) | ((np.asarray(f, np.int64) - 1) << 16)).astype(np.uint32).view(np.int32)
