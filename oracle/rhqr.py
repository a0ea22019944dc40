"""Randomized Householder QR: RHVector (Alg. 2), right-looking RHQR (Alg. 3),
left-looking RHQR (Alg. 4), block RHQR (Alg. 5), Householder QR (Sec. 2.2),
thin Q (Sec. 3.2) and recRHQR (Alg. 6).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Indices are 0-based here (column j of the code is column j+1 of the paper).
Readings of passages that are garbled or silent in the paper:

* Alg. 2, scaling line: the two choices are written without the sign of the
  pivot.  With gamma = y_j + sigma*rho (sign sigma, |gamma| = |y_j| + rho):
    scaling "B" (u_j = 1):     alpha = gamma,                  beta = |gamma|/rho
    scaling "A" (||s||^2 = 2): alpha = sqrt(rho*|gamma|),       beta = 1
  and u, s are divided by alpha.  Both give beta = 2/||s||^2.
* sign(0) = +1 (so the diagonal of R is -rho when the pivot entry is zero).
* rho = 0 (the column is already eliminated: rank-deficient W, Thm. 3.1
  hypotheses violated): identity reflector, u = e_j, s = e_j, beta = 0,
  R_jj = 0, and ``info`` records the first such column (1-based).
* Alg. 4: the sketch after the refresh is taken of the refreshed vector
  (the algorithm sketches "w"; the discussion after Alg. 2 and Thm. 3.1
  require the sketch of the updated column).  The pre-sketch of every
  column is taken once up front ("if next vector available, sketch it now").
* Prop. 3.2 writes beta_j where the new column's beta_{j+1} belongs in the
  T recursion; the recursion used is that of Alg. 4 (t_j = -beta T S^t s_j).
* Alg. 6: the triangular factor is ut(T^t S^t Z) (S = Psi U, not its head
  block); Sec. 3.3 derives it equals -T U_1^t R.
"""
import numpy as np

from .sketch import rh_sketch


def _sign(x):
    return 1.0 if x >= 0 else -1.0


def rh_vector(w, y, j, scaling="B"):
    """RHVector (Alg. 2).  ``w`` is the n-vector, ``y`` = RHSketch(w) its
    (l+m)-sketch, ``j`` the (0-based) column.  Returns u, s, sigma, rho, beta,
    alpha, ok with s = RHSketch(u) and beta = 2/||s||^2."""
    w = np.asarray(w, dtype=np.float64)
    y = np.asarray(y, dtype=np.float64)
    sigma = _sign(y[j])
    u = np.zeros_like(w)
    u[j:] = w[j:]
    s = np.zeros_like(y)
    s[j:] = y[j:]
    rho = float(np.sqrt(np.sum(s * s)))
    if rho == 0.0:
        u = np.zeros_like(w)
        u[j] = 1.0
        s = np.zeros_like(y)
        s[j] = 1.0
        return u, s, sigma, 0.0, 0.0, 1.0, False
    u[j] += sigma * rho
    s[j] += sigma * rho
    gamma = s[j]
    if scaling == "B":
        alpha = gamma
        beta = abs(gamma) / rho
    elif scaling == "A":
        alpha = float(np.sqrt(rho * abs(gamma)))
        beta = 1.0
    else:
        raise ValueError(scaling)
    return u / alpha, s / alpha, sigma, rho, beta, alpha, True


def rhqr_left(W, sk, scaling="B"):
    """Left-looking RHQR (Alg. 4).  Returns dict with U (n x m), S = Psi U
    ((l+m) x m), T (m x m upper), R (m x m upper), alpha, beta, info, and the
    pre-sketch Z = Psi W."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    L = sk.rows_out
    U = np.zeros((n, m))
    S = np.zeros((L, m))
    T = np.zeros((m, m))
    R = np.zeros((m, m))
    alpha = np.zeros(m)
    beta = np.zeros(m)
    info = 0
    Z = rh_sketch(W, sk)                       # y <- RHSketch(w_j) for every j
    for j in range(m):
        w = W[:, j].copy()
        y = Z[:, j].copy()
        if j >= 1:
            c = T[:j, :j].T @ (S[:, :j].T @ y)  # T_{j-1}^t S_{j-1}^t y
            w = w - U[:, :j] @ c                # refresh w_j
            y = rh_sketch(w, sk)                # sketch the refreshed column
        u, s, sigma, rho, b, a, ok = rh_vector(w, y, j, scaling)
        if not ok and info == 0:
            info = j + 1
        U[:, j] = u
        S[:, j] = s
        R[:j, j] = w[:j]
        R[j, j] = -sigma * rho
        T[j, j] = b
        if j >= 1:
            T[:j, j] = -b * (T[:j, :j] @ (S[:, :j].T @ s))
        alpha[j], beta[j] = a, b
    return dict(U=U, S=S, T=T, R=R, alpha=alpha, beta=beta, info=info, Z=Z)


def _left_block(M, sk, J, scaling="B"):
    """Alg. 4 on the columns of M (n x b) with pivot rows J, J+1, ...: the
    block's own U, S, T, its R columns and alpha, as Alg. 5 calls RHQR on one
    block (the block's reflectors are zero above their pivots)."""
    n, b = M.shape
    L = sk.rows_out
    U = np.zeros((n, b))
    S = np.zeros((L, b))
    T = np.zeros((b, b))
    Rc = np.zeros((J + b, b))
    info = 0
    Z = rh_sketch(M, sk)
    for c in range(b):
        j = J + c
        w = M[:, c].copy()
        y = Z[:, c].copy()
        if c >= 1:
            cc = T[:c, :c].T @ (S[:, :c].T @ y)
            w = w - U[:, :c] @ cc
            y = rh_sketch(w, sk)
        u, s, sigma, rho, beta, _, ok = rh_vector(w, y, j, scaling)
        if not ok and info == 0:
            info = j + 1
        U[:, c], S[:, c] = u, s
        Rc[:j, c] = w[:j]
        Rc[j, c] = -sigma * rho
        T[c, c] = beta
        if c >= 1:
            T[:c, c] = -beta * (T[:c, :c] @ (S[:, :c].T @ s))
    return U, S, T, Rc, info


def block_rhqr(W, sk, b, scaling="B"):
    """Block RHQR (Alg. 5): W in column blocks of b; before block j is
    factored, every earlier block k is applied to it in turn, each after a
    fresh sketch of the block (M <- M - U^(k) T^(k)^t S^(k)^t Psi M), then the
    block goes through Alg. 4 with pivots at its own columns.  Returns U, S, R
    (assembled over the blocks), the list of block T factors, and info.
    Reading: the superscripts of the update line are the earlier block's (k),
    not the current one's (j)."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    L = sk.rows_out
    U = np.zeros((n, m))
    S = np.zeros((L, m))
    R = np.zeros((m, m))
    Ts = []
    info = 0
    for J in range(0, m, b):
        nb = min(b, m - J)
        M = W[:, J:J + nb].copy()
        for k, K in enumerate(range(0, J, b)):
            Y = rh_sketch(M, sk)
            kb = Ts[k].shape[0]
            M = M - U[:, K:K + kb] @ (Ts[k].T @ (S[:, K:K + kb].T @ Y))
        Ub, Sb, Tb, Rc, ib = _left_block(M, sk, J, scaling)
        if ib and not info:
            info = ib
        U[:, J:J + nb], S[:, J:J + nb] = Ub, Sb
        R[:J + nb, J:J + nb] = Rc
        Ts.append(Tb)
    return dict(U=U, S=S, R=R, Ts=Ts, info=info)


def rhqr_right(W, sk, scaling="B"):
    """Right-looking RHQR (Alg. 3).  Returns dict with U, S, R, beta."""
    W = np.array(W, dtype=np.float64, copy=True)
    n, m = W.shape
    L = sk.rows_out
    U = np.zeros((n, m))
    S = np.zeros((L, m))
    R = np.zeros((m, m))
    beta = np.zeros(m)
    for j in range(m):
        w = W[:, j].copy()
        Yall = rh_sketch(W[:, j:], sk)          # sketch of the m-j+1 trailing columns
        y, Y = Yall[:, 0], Yall[:, 1:]
        u, s, sigma, rho, b, _, _ = rh_vector(w, y, j, scaling)
        U[:, j], S[:, j], beta[j] = u, s, b
        R[:j, j] = w[:j]
        R[j, j] = -sigma * rho
        if j < m - 1:
            W[:, j + 1:] = W[:, j + 1:] - b * np.outer(u, s @ Y)
    return dict(U=U, S=S, R=R, beta=beta)


def hqr(Z):
    """Deterministic Householder QR of Z (Sec. 2.2), right-looking, with the
    sign choice of eq. (sumup) and reflectors scaled to a unit pivot entry.
    Returns V (Householder vectors), T (compact-WY factor built by the
    recursion T_{j+1} = [[T_j, -beta T_j V_j^t v_{j+1}], [0, beta]]), R."""
    A = np.array(Z, dtype=np.float64, copy=True)
    p, m = A.shape
    V = np.zeros((p, m))
    T = np.zeros((m, m))
    R = np.zeros((m, m))
    for j in range(m):
        x = A[j:, j]
        rho = float(np.sqrt(np.sum(x * x)))
        sigma = _sign(x[0])
        if rho == 0.0:
            v = np.zeros(p)
            v[j] = 1.0
            b = 0.0
        else:
            gamma = x[0] + sigma * rho
            v = np.zeros(p)
            v[j] = 1.0
            v[j + 1:] = x[1:] / gamma
            b = abs(gamma) / rho               # = 2 / ||v||^2
        V[:, j] = v
        R[:j, j] = A[:j, j]
        R[j, j] = -sigma * rho
        # apply P(v) = I - b v v^t to the trailing columns
        if j < m - 1:
            A[:, j + 1:] -= b * np.outer(v, v @ A[:, j + 1:])
        T[j, j] = b
        if j >= 1:
            T[:j, j] = -b * (T[:j, :j] @ (V[:, :j].T @ v))
    return V, T, R


def thin_q(U, T, m):
    """Thin Q factor Q = [I_m; 0] - U T U_{1:m,1:m}^t (Sec. 3.2)."""
    n = U.shape[0]
    E = np.zeros((n, m))
    E[:m, :m] = np.eye(m)
    return E - U @ (T @ U[:m, :m].T)


def _forward_subst_right(B, M):
    """Solve X M = B for X with M upper triangular, column by column:
    x_j = (b_j - X_{:,<j} M_{<j,j}) / M_jj (the explicit recursion of Sec. 3.3)."""
    X = np.zeros_like(B)
    for j in range(M.shape[0]):
        X[:, j] = (B[:, j] - X[:, :j] @ M[:j, j]) / M[j, j]
    return X


def rec_rhqr(W, sk, mode="M"):
    """recRHQR (Alg. 6).  mode "M": U_2 = W_2 ut(T^t S^t Z)^{-1}, U = [S_{1:m}; U_2],
    Q from the thin-Q formula.  mode "R" (randomized Cholesky QR, Sec. 8):
    Q = W R^{-1} with U, T, S from the sketch-space QR."""
    W = np.asarray(W, dtype=np.float64)
    n, m = W.shape
    Z = rh_sketch(W, sk)                      # single synchronisation
    S, T, R = hqr(Z)
    Y = S[:m, :m]
    M = np.triu(T.T @ S.T @ Z)
    if mode == "M":
        X = _forward_subst_right(W[m:], M)
        U = np.concatenate([Y, X], axis=0)
        Q = thin_q(U, T, m)
    elif mode == "R":
        Q = _forward_subst_right(W, R)
        U = None
    else:
        raise ValueError(mode)
    return dict(U=U, S=S, T=T, R=R, M=M, Q=Q, Z=Z)
