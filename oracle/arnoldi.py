"""RHQR-Arnoldi (Alg. 7) and RHQR-GMRES (Alg. 8), restarted.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Readings of garbled passages:

* Alg. 7 runs j up to m+1, so the sketch Psi keeps k = m+1 head rows
  (Omega acts on the last n-m-1 rows).
* Alg. 7, first sketch inside the loop: the vector sketched is w = A q_j
  (the algorithm writes the sketch of z).
* Alg. 8: the right-hand side of the small least-squares problem is
  beta e_1 with beta = (h_0)_1 = -sigma_1 rho_1 (eq. sumup); the solution is
  x = x_0 + Q_m y = x_0 + [y; 0] - U T S^t Psi [y; 0], where the head rows of S
  are those of U.
"""
import numpy as np

from .rhqr import rh_vector
from .sketch import rh_sketch


def rhqr_arnoldi(A, r0, sk, m):
    """Alg. 7 with starting residual r0 = b - A x0.  ``sk`` has m+1 head rows.
    Returns dict(U, S, T, H ((m+1) x m), h0, Q (explicit q_1..q_{m+1}))."""
    n = r0.shape[0]
    k = m + 1
    assert sk.m == k
    L = sk.rows_out
    U = np.zeros((n, k))
    S = np.zeros((L, k))
    T = np.zeros((k, k))
    Hfull = np.zeros((k, k))        # column j holds h_j (j = 0..m)
    Q = np.zeros((n, k))
    w = np.asarray(r0, dtype=np.float64).copy()
    z = rh_sketch(w, sk)
    for j in range(k):              # paper's j = 1..m+1
        u, s, sigma, rho, b, _, _ = rh_vector(w, z, j)
        U[:, j], S[:, j] = u, s
        Hfull[:j, j] = w[:j]
        Hfull[j, j] = -sigma * rho
        T[j, j] = b
        if j >= 1:
            T[:j, j] = -b * (T[:j, :j] @ (S[:, :j].T @ s))
        if j < m or j == m:
            # q_{j+1} = e_{j+1} - U_j T_j S_j^t e_{j+1} (0-based column j)
            e = np.zeros(n)
            e[j] = 1.0
            q = e - U[:, :j + 1] @ (T[:j + 1, :j + 1] @ S[j, :j + 1])
            Q[:, j] = q
        if j < m:
            w = A @ q
            z = rh_sketch(w, sk)
            w = w - U[:, :j + 1] @ (T[:j + 1, :j + 1].T @ (S[:, :j + 1].T @ z))
            z = rh_sketch(w, sk)
    H = Hfull[:, 1:]                 # h_1..h_m, first m+1 rows
    return dict(U=U, S=S, T=T, H=H, h0=Hfull[:, 0], Q=Q)


def rhqr_gmres_cycle(A, b, x0, sk, m):
    """One cycle of Alg. 8: returns x_m minimising ||Psi (b - A x)|| over
    x0 + K_m(A, r0)."""
    r0 = b - A @ x0
    arn = rhqr_arnoldi(A, r0, sk, m)
    beta = arn["h0"][0]
    rhs = np.zeros(m + 1)
    rhs[0] = beta
    y = np.linalg.lstsq(arn["H"], rhs, rcond=None)[0]
    U, T, S = arn["U"][:, :m], arn["T"][:m, :m], arn["S"][:, :m]
    ypad = np.zeros(b.shape[0])
    ypad[:m] = y
    x = x0 + ypad - U @ (T @ (S[:m].T @ y))
    return x, arn, y


def rhqr_gmres(A, b, sk, m, tol=1e-6, max_cycles=50, x0=None):
    """Restarted RHQR-GMRES(m); the true residual is recomputed in float64 at
    each restart.  Returns x and the list of relative residuals per cycle."""
    x = np.zeros_like(b) if x0 is None else x0.copy()
    hist = []
    nb = np.linalg.norm(b)
    for _ in range(max_cycles):
        x, _, _ = rhqr_gmres_cycle(A, b, x, sk, m)
        rel = np.linalg.norm(b - A @ x) / nb
        hist.append(rel)
        if rel <= tol:
            break
    return x, hist
