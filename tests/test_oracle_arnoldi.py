"""Pins of the oracle's RHQR-Arnoldi / RHQR-GMRES (Sec. 5): the Arnoldi
relation (eq. arnoldirelation), sketch orthonormality of the Krylov basis
(Thm. 3.1 applied to the Arnoldi vectors), and the Psi-norm optimality of
Prop. rgmresopti checked by brute-force least squares on an explicit Krylov
basis."""
import numpy as np
import scipy.sparse as sp

from oracle import arnoldi, sketch
from paper_2405_10923_amd.inputs import convdiff_csr


def _operator(nx):
    indptr, indices, values, n = convdiff_csr(nx)
    return sp.csr_matrix((values, indices, indptr), shape=(n, n)), n


def test_arnoldi_relation_and_sketch_orthonormality():
    A, n = _operator(20)
    m = 12
    sk = sketch.Sketch(sketch.SRHT, n, m + 1, 60, seed=3)
    r0 = np.ones(n)
    arn = arnoldi.rhqr_arnoldi(A, r0, sk, m)
    Q = arn["Q"]
    lhs = A @ Q[:, :m]
    rhs = Q @ arn["H"]
    assert np.linalg.norm(lhs - rhs) <= 1e-13 * np.linalg.norm(lhs)
    PQ = sketch.rh_sketch(Q, sk)
    assert np.linalg.norm(PQ.T @ PQ - np.eye(m + 1), 2) < 1e-12
    # q_1 is a multiple of r0 with factor 1/(h_0)_1
    assert np.allclose(Q[:, 0] * arn["h0"][0], r0, atol=1e-12)
    # H is upper Hessenberg
    assert np.all(np.tril(arn["H"], -2) == 0)


def test_gmres_cycle_minimises_sketched_residual():
    A, n = _operator(16)
    m = 10
    sk = sketch.Sketch(sketch.SRHT, n, m + 1, 50, seed=5)
    b = np.ones(n)
    x0 = np.random.default_rng(0).standard_normal(n) * 0.1
    x, arn, y = arnoldi.rhqr_gmres_cycle(A, b, x0, sk, m)
    r0 = b - A @ x0
    # brute force over an explicit (orthonormalised) Krylov basis
    K = np.zeros((n, m))
    v = r0 / np.linalg.norm(r0)
    for i in range(m):
        K[:, i] = v
        v = A @ v
        v -= K[:, :i + 1] @ (K[:, :i + 1].T @ v)
        v /= np.linalg.norm(v)
    PsiAK = sketch.rh_sketch(A @ K, sk)
    c = np.linalg.lstsq(PsiAK, sketch.rh_sketch(r0, sk), rcond=None)[0]
    best = np.linalg.norm(sketch.rh_sketch(r0 - A @ (K @ c), sk))
    got = np.linalg.norm(sketch.rh_sketch(b - A @ x, sk))
    assert abs(got - best) <= 1e-9 * np.linalg.norm(sketch.rh_sketch(r0, sk))
    # x - x0 lies in the Krylov space
    d = x - x0
    assert np.linalg.norm(d - K @ (K.T @ d)) <= 1e-9 * np.linalg.norm(d)


def test_restarted_gmres_converges():
    A, n = _operator(24)
    m = 20
    sk = sketch.Sketch(sketch.SRHT, n, m + 1, 80, seed=1)
    b = np.ones(n)
    x, hist = arnoldi.rhqr_gmres(A, b, sk, m, tol=1e-8, max_cycles=40)
    assert hist[-1] <= 1e-8
    assert all(h2 <= h1 * (1 + 1e-12) for h1, h2 in zip(hist, hist[1:]))
