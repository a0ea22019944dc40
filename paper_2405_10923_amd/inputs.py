"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module builds test matrices and operators only; it holds none of the
factorization's arithmetic.

* ``synthetic_matrix``: W = G diag(s) V with G iid N(0,1) (n x m), singular values
  s_i = 10^(-kappa * i / (m-1)) logarithmically spaced from 1 to 10^-kappa,
  and V a Haar-distributed orthogonal m x m matrix (QR of a Gaussian matrix
  with the signs of diag(R) moved into Q).
* ``cm_matrix``: the parametric-function matrix C_m of Sec. 8,
  C_{i,j} = f((i-1)/(n-1), (j-1)/(m-1)), f(x, mu) = sin(10(mu+x)) /
  (cos(100(mu-x)) + 1.1).
* ``convdiff_csr``: a 5-point upwind convection-diffusion operator in CSR
  form (the sparse operator of the GMRES workload).
"""
import numpy as np


def haar_orthogonal(m, rng):
    A = rng.standard_normal((m, m))
    Q, R = np.linalg.qr(A)
    return Q * np.sign(np.diag(R))


def singular_values(m, kappa_log10):
    if m == 1:
        return np.ones(1)
    return 10.0 ** (-float(kappa_log10) * np.arange(m) / (m - 1))


def synthetic_matrix(n, m, kappa_log10, seed=0):
    """float64 n x m matrix with condition number 10^kappa_log10 (numpy RNG)."""
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((n, m))
    V = haar_orthogonal(m, rng)
    s = singular_values(m, kappa_log10)
    return np.asfortranarray((G * s) @ V)


def synthetic_matrix_torch(n, m, kappa_log10, seed=0, device="cuda"):
    """Same construction with G drawn by torch on ``device`` (large sizes).
    Returned as a column-major (n x m) float64 torch tensor (a transposed view
    of an m x n row-major buffer)."""
    import torch
    gen = torch.Generator(device=device)
    gen.manual_seed(int(seed))
    rng = np.random.default_rng(seed)
    V = haar_orthogonal(m, rng)
    s = singular_values(m, kappa_log10)
    B = torch.from_numpy((s[:, None] * V).T.copy()).to(device)   # (m x m) = (diag(s) V)^t
    Wt = torch.empty((m, n), dtype=torch.float64, device=device)
    chunk = 1 << 20
    for r0 in range(0, n, chunk):
        r1 = min(n, r0 + chunk)
        Gt = torch.randn((m, r1 - r0), dtype=torch.float64, device=device, generator=gen)
        Wt[:, r0:r1] = B @ Gt   # (W^t)[:, rows] = (diag(s)V)^t G^t
    return Wt.t()


def cm_matrix(n, m):
    x = np.arange(n) / (n - 1)
    mu = np.arange(m) / (m - 1)
    X, MU = np.meshgrid(x, mu, indexing="ij")
    return np.asfortranarray(np.sin(10 * (MU + X)) / (np.cos(100 * (MU - X)) + 1.1))


def convdiff_csr(nx, peclet=10.0):
    """-Laplace(u) + b . grad(u) on the unit square, b = (beta, beta), on an
    nx x nx interior grid (h = 1/(nx+1)), homogeneous Dirichlet boundary,
    first-order upwind convection, rows scaled by h^2.  The cell Peclet number
    beta*h/2 equals ``peclet``.  Unknowns in lexicographic order (x fastest).
    Returns (indptr int64, indices int32, values float64, n)."""
    n = nx * nx
    # per row: diag 4 + beta*h*2 ; west/south -1 - beta*h ; east/north -1
    bh = 2.0 * peclet
    diag = 4.0 + 2.0 * bh
    west = -1.0 - bh
    east = -1.0
    idx = np.arange(n)
    ix = idx % nx
    iy = idx // nx
    cols, vals = [], []
    for dx, dy, v in ((0, -1, west), (-1, 0, west), (0, 0, diag), (1, 0, east), (0, 1, east)):
        ok = (ix + dx >= 0) & (ix + dx < nx) & (iy + dy >= 0) & (iy + dy < nx)
        c = np.where(ok, idx + dx + dy * nx, -1)
        cols.append(c)
        vals.append(np.where(ok, v, 0.0))
    C = np.stack(cols, axis=1)
    Vv = np.stack(vals, axis=1)
    keep = C >= 0
    counts = keep.sum(axis=1)
    indptr = np.zeros(n + 1, dtype=np.int64)
    np.cumsum(counts, out=indptr[1:])
    indices = C[keep].astype(np.int32)
    values = Vv[keep].astype(np.float64)
    return indptr, indices, values, n
