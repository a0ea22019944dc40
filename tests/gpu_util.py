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


def psi_apply_torch(osketch, X, chunk=32):
    """Psi X for the oracle's draw of Psi (its signs and sampled rows, or its
    Omega), evaluated with plain torch operations on X's device in float64:
    the same steps as the oracle's RHSketch (head rows copied; tail rows
    zero-padded to N, scaled by sqrt(N/l), sign-flipped, Walsh-Hadamard
    transformed by butterflies, divided by sqrt(N), sampled).  Test-side
    evaluation of the oracle's definition at sizes where numpy is too slow; it
    shares nothing with the library."""
    import math
    import torch
    n, k = X.shape
    m, l = osketch.m, osketch.l
    dev = X.device
    out = torch.empty((m + l, k), dtype=torch.float64, device=dev)
    out[:m] = X[:m].to(torch.float64)
    if osketch.kind == "gauss":
        om = torch.from_numpy(np.ascontiguousarray(osketch.omega)).to(dev)
        for c0 in range(0, k, chunk):
            c1 = min(k, c0 + chunk)
            out[m:, c0:c1] = om @ X[m:, c0:c1].to(torch.float64)
        return out
    N = osketch.N
    signs = torch.from_numpy(osketch.signs).to(dev)
    rows = torch.from_numpy(osketch.rows).to(dev)
    for c0 in range(0, k, chunk):
        c1 = min(k, c0 + chunk)
        kc = c1 - c0
        v = torch.zeros((N, kc), dtype=torch.float64, device=dev)
        v[m:n] = X[m:, c0:c1].to(torch.float64)
        v *= math.sqrt(N / l)
        v *= signs[:, None]
        h = 1
        while h < N:
            w = v.view(N // (2 * h), 2, h, kc)
            a = w[:, 0].clone()
            b = w[:, 1]
            w[:, 0] = a + b
            w[:, 1] = a - b
            h *= 2
        v /= math.sqrt(N)
        out[m:, c0:c1] = v[rows]
        del v
    return out


def cond_gram(Q):
    """cond(Q) from the eigenvalues of Q^t Q, formed in float64 by torch."""
    import torch
    G = Q.to(torch.float64)
    G = (G.t() @ G).cpu().numpy()
    ev = np.linalg.eigvalsh(G)
    return float(np.sqrt(ev[-1] / ev[0])) if ev[0] > 0 else float("inf")


def orth_err(PQ):
    """||(Psi Q)^t (Psi Q) - I||_2 in float64."""
    import torch
    P = PQ.to(torch.float64)
    G = (P.t() @ P).cpu().numpy()
    return float(np.linalg.norm(G - np.eye(G.shape[0]), 2))
