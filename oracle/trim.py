"""trimRHQR: randomized reflectors with partial sketching (Sec. 7):
trimRHVector (Alg. 10), right-looking trimRHQR (Alg. 11), left-looking
trimRHQR (Alg. 12), the thin Q factor and the two compact forms.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Here Omega (l x n) sketches every row of W, so l may be smaller than m.
The reflector that eliminates below row j sketches with
Psi_j = [I_{j-1} 0; 0 Omega_{j:n}] (eq. psij); for a vector u whose first
j-1 entries vanish it is H(u, Omega, j) = I - 2/||Omega u||^2 u (Omega u)^t
[0 Omega_{j:n}] (eq. rhousebisbis).  It eliminates only if the columns
Omega e_1 .. Omega e_m have unit norm, as for the SRHT (every entry +-l^-1/2).
Indices are 0-based (column j here is the paper's j+1).

Readings of garbled passages:
* Alg. 10, scaling line: "alpha as the first entry of v'" reads as the
  unit-pivot scaling alpha = 1 / v_j (v divided by its pivot entry, like
  Alg. 2's scaling B), the other choice being sqrt 2 / ||v'||; in both cases
  beta = 2 / ||s||^2 with s the scaled sketch Omega v (beta = 1 for the
  second choice).
* Alg. 10 needs the sketch of v = w' + sigma rho e_j; it is formed from the
  sketch of w' and the sketch of e_j (no extra synchronisation), and the
  sketch of w' from that of the refreshed w minus its first j entries' terms.
* Alg. 12: "T_{1:j-1,1:j-1} S_j^t s_j" reads S_{j-1}^t s_j (the earlier
  reflectors), and both T recursions use the new column's beta (as for
  Alg. 4).
* Prop. (Qmbis) writes beta_{j} in the bottom-right entry of T~_{j+1}; the
  new column's beta is used.
"""
import numpy as np

from .sketch import SRHT, fwht, next_pow2, srht_rows, srht_signs


class FullSketch:
    """Omega of Sec. 7: an SRHT of R^N (N = 2^ceil(log2 n)) applied to all n
    rows (coordinates 0..n-1; padding zero), with the draw of Sec. 2.3's SRHT
    (the same generator streams as the structured sketch)."""

    def __init__(self, n, l, seed=0):
        self.n, self.l, self.seed = int(n), int(l), seed
        self.N = next_pow2(self.n)
        self.signs = srht_signs(seed, self.N)
        self.rows = srht_rows(seed, self.N, self.l)

    def apply(self, X):
        X = np.asarray(X, dtype=np.float64)
        N, n, l = self.N, self.n, self.l
        v = np.zeros((N,) + X.shape[1:])
        v[:n] = X
        v = np.sqrt(N / l) * v
        v = self.signs.reshape((N,) + (1,) * (v.ndim - 1)) * v
        v = fwht(v)
        v = v / np.sqrt(N)
        return v[self.rows]


def _sign(x):
    return 1.0 if x >= 0 else -1.0


def trim_vector(w, zw, E, j, scaling="B"):
    """trimRHVector (Alg. 10) for the vector w (n entries; only rows >= j
    matter) given zw = Omega w and E = Omega[:, :j+1] (the sketches of e_0..e_j).
    Returns u (zeros above row j), s = Omega u, sigma, rho, beta, alpha."""
    n = w.shape[0]
    # sketch of w' = (0_{j}; w_{j:})
    zp = zw - E[:, :j] @ w[:j]
    rho = float(np.linalg.norm(zp))
    sigma = _sign(w[j])
    v = np.zeros(n)
    v[j:] = w[j:]
    v[j] += sigma * rho
    s = zp + sigma * rho * E[:, j]             # Omega v
    if scaling == "B":
        alpha = v[j]
        u, s = v / alpha, s / alpha
        beta = 2.0 / float(s @ s)
    else:
        alpha = np.sqrt(2.0) / float(np.linalg.norm(s))
        u, s = v * alpha, s * alpha
        beta = 1.0
    return u, s, sigma, rho, beta, alpha


def trim_rhqr_right(W, om, scaling="B"):
    """Right-looking trimRHQR (Alg. 11): reflector j is applied to the
    trailing columns right after it is formed, with the sketch of their rows
    from j on.  Returns U, S = Omega U, R, beta."""
    W = np.array(W, dtype=np.float64, copy=True)
    n, m = W.shape
    l = om.l
    E = om.apply(np.eye(n, m))
    U = np.zeros((n, m))
    S = np.zeros((l, m))
    R = np.zeros((m, m))
    beta = np.zeros(m)
    for j in range(m):
        w = W[:, j].copy()
        u, s, sigma, rho, b, _ = trim_vector(w, om.apply(w), E, j, scaling)
        U[:, j], S[:, j], beta[j] = u, s, b
        R[:j, j] = w[:j]
        R[j, j] = -sigma * rho
        if j + 1 < m:
            Xt = W[:, j + 1:].copy()
            Xt[:j] = 0.0                          # [0 Omega_{j:n}] W_{:, j+1:}
            X = om.apply(Xt)
            W[:, j + 1:] -= b * np.outer(u, s @ X)
    return dict(U=U, S=S, R=R, beta=beta)


def trim_rhqr_left(W, om, scaling="B"):
    """Left-looking trimRHQR (Alg. 12).  Returns U, S = Omega U, T, Tt (the
    T~ of the left-wise product), R, the slt((Omega U)^t Omega) block K
    (K[p, i] = <Omega u_p, Omega e_i>, i < p, i < m), beta, alpha."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    l = om.l
    E = om.apply(np.eye(n, m))               # sketches of e_0 .. e_{m-1}
    U = np.zeros((n, m))
    S = np.zeros((l, m))
    T = np.zeros((m, m))
    Tt = np.zeros((m, m))
    R = np.zeros((m, m))
    K = np.zeros((m, m))
    beta = np.zeros(m)
    alpha = np.zeros(m)
    Zw = om.apply(W)
    for j in range(m):
        w = W[:, j].copy()
        if j >= 1:
            # ut((Omega U)^t Omega) w = (Omega U)^t Omega w - slt(...) w
            a = S[:, :j].T @ Zw[:, j] - K[:j, :j] @ w[:j]
            w = w - U[:, :j] @ (Tt[:j, :j].T @ a)
        u, s, sigma, rho, b, al = trim_vector(w, om.apply(w), E, j, scaling)
        U[:, j], S[:, j], beta[j], alpha[j] = u, s, b, al
        R[:j, j] = w[:j]
        R[j, j] = -sigma * rho
        T[j, j] = b
        Tt[j, j] = b
        if j >= 1:
            T[:j, j] = -b * (T[:j, :j] @ (S[:, :j].T @ s))
            Sp = S[:, :j] - E[:, :j] @ U[:j, :j]   # [0 Omega_{j:n}] U_{j-1}
            Tt[:j, j] = -b * (Tt[:j, :j] @ (Sp.T @ s))
        K[j, :j] = s @ E[:, :j]
    return dict(U=U, S=S, T=T, Tt=Tt, R=R, K=K, beta=beta, alpha=alpha, E=E)


def trim_ut(S, E, m):
    """The m x m block ut((Omega U)^t Omega)[I_m; 0]: entry (p, i) =
    <Omega u_p, Omega e_i> for i >= p, zero below the diagonal."""
    return np.triu(S.T @ E[:, :m])


def trim_thin_q(U, T, S, E, m):
    """Q = H_1 ... H_m [I_m; 0] = [I_m; 0] - U T ut((Omega U)^t Omega)[I_m; 0]
    (eq. compactrightbis)."""
    n = U.shape[0]
    I = np.zeros((n, m))
    I[:m, :m] = np.eye(m)
    return I - U @ (T @ trim_ut(S, E, m))
