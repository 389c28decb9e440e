"""Helpers shared by the GPU tests (no method arithmetic here)."""
import sys

import numpy as np


def torch_cuda():
    import torch
    if not torch.cuda.is_available():
        import pytest
        pytest.skip("no GPU")
    return torch


def dev(a):
    torch = torch_cuda()
    return torch.from_numpy(np.ascontiguousarray(a)).to("cuda")


def host(t):
    return t.detach().cpu().numpy()


def rel(a, b):
    """max |a - b| / max |b|"""
    return float(np.abs(a - b).max() / max(np.abs(b).max(), 1e-300))


def say(*args):
    print(*args, flush=True)
    sys.stdout.flush()
