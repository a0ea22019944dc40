"""Helpers shared by the GPU tests (no method arithmetic here)."""
import numpy as np
import pytest


def cuda_or_skip():
    torch = pytest.importorskip("torch")
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    return torch


def to_gpu(A, dtype=None):
    """numpy (r x c) -> column-major torch tensor on cuda:0."""
    import torch
    A = np.asarray(A)
    if A.ndim == 1:
        A = A.reshape(-1, 1)
    dt = dtype or torch.float64
    t = torch.empty((A.shape[1], A.shape[0]), dtype=dt, device="cuda").t()
    t.copy_(torch.from_numpy(np.ascontiguousarray(A)).to(dt))
    return t


def to_np(t):
    import torch
    return t.detach().to(torch.float64).cpu().numpy()


def rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    d = np.max(np.abs(a - b))
    s = max(np.max(np.abs(b)), 1e-300)
    return d / s


def log(msg):
    print(msg, flush=True)
