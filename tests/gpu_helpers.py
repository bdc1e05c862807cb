"""Shared helpers of the GPU parity tests (not collected by pytest)."""

import sys

import numpy as np


def say(*args):
    """Name the case before each GPU step (flushed, so a fault still shows it)."""
    print("[gpu-case]", *args, file=sys.stderr, flush=True)


def torch_cuda():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def to_dev(x):
    torch = torch_cuda()
    return torch.as_tensor(np.ascontiguousarray(x, dtype=np.float64), device="cuda:0")


def principal_cosines(U, V):
    """Cosines of the principal angles between span(U) and span(V)."""
    Qu = np.linalg.qr(U)[0]
    Qv = np.linalg.qr(V)[0]
    return np.linalg.svd(Qu.T @ Qv, compute_uv=False)
