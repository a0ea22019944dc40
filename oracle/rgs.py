"""BLAS2-RGS (Alg. 9, Sec. 6) and plain randomized Gram-Schmidt.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Sec. 6 obtains BLAS2-RGS as left-looking RHQR of [0_{m x m}; W] with
Psi = [I_m 0; 0 Omega], Omega acting on the n rows of W.  Here the sketch
object describes that Psi: its row count is n + m and its head m, so its
Omega applies to W itself.

Readings:
* the line "rho = ||Omega z||" sketches twice by a typo: rho = ||z|| with
  z = Omega w (the norm of the sketch of the refreshed column), and "s" in
  "s_j <- rho^-1 s" is that z;
* T_{j-1} in the refresh is the leading (j-1) x (j-1) block of T; every
  beta equals 1 (the sketched norm of [e_j; -q_j] is sqrt 2);
* the optional last line (Q <- Q T) is not applied: Q is returned as the
  loop forms it.
"""
import numpy as np


def blas2_rgs(W, sk):
    """Alg. 9.  ``sk`` has n + m rows and head m (W is n x m).  Returns dict
    Q (n x m), R (m x m upper, positive diagonal), T (m x m upper, unit
    diagonal), S = Omega Q (l x m)."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    assert sk.n == n + m and sk.m == m
    l = sk.l
    Q = np.zeros((n, m))
    S = np.zeros((l, m))
    T = np.zeros((m, m))
    R = np.zeros((m, m))
    for j in range(m):
        w = W[:, j].copy()
        r = np.zeros(0)
        if j >= 1:
            z = sk.omega_apply(w)
            r = T[:j, :j].T @ (S[:, :j].T @ z)
            w = w - Q[:, :j] @ r
        z = sk.omega_apply(w)
        rho = float(np.sqrt(np.sum(z * z)))
        Q[:, j] = w / rho
        S[:, j] = z / rho
        R[:j, j] = r
        R[j, j] = rho
        T[j, j] = 1.0
        if j >= 1:
            T[:j, j] = -(T[:j, :j] @ (S[:, :j].T @ S[:, j]))
    return dict(Q=Q, R=R, T=T, S=S)


def rgs(W, sk):
    """Randomized Gram-Schmidt, the classical-Gram-Schmidt form Sec. 6 proves
    BLAS2-RGS equivalent to: q~_j = w_j - Q (Omega Q)^t Omega w_j,
    q_j = q~_j / ||Omega q~_j||, R_{:j, j} = (Omega Q)^t Omega w_j,
    R_jj = ||Omega q~_j||."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    Q = np.zeros((n, m))
    R = np.zeros((m, m))
    for j in range(m):
        w = W[:, j]
        P = sk.omega_apply(Q[:, :j])
        r = P.T @ sk.omega_apply(w)
        qt = w - Q[:, :j] @ r
        rho = float(np.linalg.norm(sk.omega_apply(qt)))
        Q[:, j] = qt / rho
        R[:j, j] = r
        R[j, j] = rho
    return dict(Q=Q, R=R)
