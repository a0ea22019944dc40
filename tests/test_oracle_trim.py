"""Pins of the oracle's trimRHQR (Sec. 7, Alg. 10-12).

* Brute force: the reflectors H(u_j, Omega, j) = I - 2/||Psi_j u||^2 u
  (Psi_j u)^t Psi_j built as dense matrices from eq. (psij) on a small n
  eliminate W column by column: H_m ... H_1 W = [R; 0].
* Alg. 11 (right-looking) and Alg. 12 (left-looking) give the same U, S, R.
* The compact forms of Prop. (Qbis) and (Qmbis): W = (I - U T ut) [R; 0]
  and (I - U T~^t ut) W = [R; 0], ut = ut((Omega U)^t Omega) formed densely.
* The Woodbury identities of Props. (woodburrybis) and (deltawoodburry):
  T^-1 + T^-t = (Omega U)^t Omega U and T~^t = -[T^-1 - ut U]^-1.
* The SRHT's columns are unit vectors (the hypothesis the elimination needs),
  and the method works with fewer sketch rows than columns (l < m).
* A plausible mistake (forgetting the slt correction, i.e. applying
  (Omega U)^t Omega instead of its upper-triangular part) is caught."""
import numpy as np
import pytest

from oracle import trim
from paper_2405_10923_amd.inputs import synthetic_matrix


def _dense_omega(om, n):
    return om.apply(np.eye(n))


def _ut_dense(S, Od):
    """ut((Omega U)^t Omega): entry (p, i) kept for i >= p."""
    A = S.T @ Od
    return np.triu(A)


@pytest.mark.parametrize("n,m,l", [(64, 6, 16), (100, 10, 8), (128, 12, 40)])
def test_dense_reflectors_eliminate(n, m, l):
    W = synthetic_matrix(n, m, 2, seed=n)
    om = trim.FullSketch(n, l, seed=3)
    Od = _dense_omega(om, n)
    assert np.allclose(np.linalg.norm(Od, axis=0), 1.0, rtol=0, atol=1e-14)
    r = trim.trim_rhqr_left(W, om)
    X = W.copy()
    for j in range(m):
        u = r["U"][:, j]
        assert np.all(u[:j] == 0.0)
        Psi = np.zeros((l + j, n))
        Psi[:j, :j] = np.eye(j)
        Psi[j:, j:] = Od[:, j:]
        pu = Psi @ u
        H = np.eye(n) - (2.0 / (pu @ pu)) * np.outer(u, pu) @ Psi
        X = H @ X
    Rb = np.zeros((n, m))
    Rb[:m] = r["R"]
    assert np.max(np.abs(X - Rb)) <= 1e-12 * np.max(np.abs(W))


@pytest.mark.parametrize("scaling", ["B", "A"])
def test_left_equals_right_and_compact_forms(scaling):
    n, m, l = 200, 12, 30
    W = synthetic_matrix(n, m, 3, seed=2)
    om = trim.FullSketch(n, l, seed=5)
    Od = _dense_omega(om, n)
    lf = trim.trim_rhqr_left(W, om, scaling)
    rt = trim.trim_rhqr_right(W, om, scaling)
    for k in ("U", "S", "R"):
        assert np.max(np.abs(lf[k] - rt[k])) <= 1e-12 * np.max(np.abs(rt[k])), k
    U, S, T, Tt, R = lf["U"], lf["S"], lf["T"], lf["Tt"], lf["R"]
    assert np.allclose(Od @ U, S, rtol=0, atol=1e-13)
    ut = _ut_dense(S, Od)
    Rb = np.zeros((n, m))
    Rb[:m] = R
    assert np.linalg.norm(W - (Rb - U @ (T @ (ut @ Rb)))) <= 1e-13 * np.linalg.norm(W)
    assert np.linalg.norm((W - U @ (Tt.T @ (ut @ W))) - Rb) <= 1e-13 * np.linalg.norm(W)
    Ti = np.linalg.inv(T)
    assert np.allclose(Ti + Ti.T, S.T @ S, rtol=0, atol=1e-12)
    assert np.allclose(Tt.T, -np.linalg.inv(Ti - ut @ U), rtol=0, atol=1e-12)
    # K holds slt((Omega U)^t Omega)'s first m columns
    A = S.T @ Od[:, :m]
    assert np.allclose(lf["K"], np.tril(A, -1), rtol=0, atol=1e-14)
    # thin Q of the compact form
    Q = trim.trim_thin_q(U, T, S, lf["E"], m)
    assert np.linalg.norm(W - Q @ R) <= 1e-13 * np.linalg.norm(W)


def test_fewer_sketch_rows_than_columns():
    """l < m (Sec. 7, Figs. perf64bis / perf32bis): the factorization stays
    accurate (Q is no longer sketch-orthonormal, so its conditioning depends
    on l and is not pinned)."""
    n, m = 4096, 48
    W = synthetic_matrix(n, m, 6, seed=7)
    for l in (16, 32):
        om = trim.FullSketch(n, l, seed=1)
        r = trim.trim_rhqr_left(W, om)
        Q = trim.trim_thin_q(r["U"], r["T"], r["S"], r["E"], m)
        assert np.linalg.norm(W - Q @ r["R"]) <= 1e-12 * np.linalg.norm(W)


def test_mutation_missing_slt_correction_is_caught():
    n, m, l = 200, 10, 30
    W = synthetic_matrix(n, m, 2, seed=2)
    om = trim.FullSketch(n, l, seed=5)
    good = trim.trim_rhqr_left(W, om)
    E = good["E"]
    U = np.zeros((n, m)); S = np.zeros((l, m)); Tt = np.zeros((m, m)); R = np.zeros((m, m))
    for j in range(m):
        w = W[:, j].copy()
        if j:
            a = S[:, :j].T @ om.apply(W[:, j])          # slt correction forgotten
            w = w - U[:, :j] @ (Tt[:j, :j].T @ a)
        u, s, sigma, rho, b, _ = trim.trim_vector(w, om.apply(w), E, j)
        U[:, j], S[:, j] = u, s
        R[:j, j], R[j, j] = w[:j], -sigma * rho
        Tt[j, j] = b
        if j:
            Sp = S[:, :j] - E[:, :j] @ U[:j, :j]
            Tt[:j, j] = -b * (Tt[:j, :j] @ (Sp.T @ s))
    assert np.max(np.abs(R - good["R"])) > 1e-6 * np.max(np.abs(good["R"]))
