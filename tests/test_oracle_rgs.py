"""Pins of the oracle's BLAS2-RGS (Alg. 9, Sec. 6).

* Sec. 6 derives it as left-looking RHQR of [0; W]: the oracle's RHQR of the
  zero-topped matrix must give the same factors (Householder vectors [e_j;
  q_j] with the pivot sign never flipped, so U's tail is Q, R is the negated
  RHQR R, T the same T, S the tail of RHQR's S);
* the proposition of Sec. 6: it equals randomized Gram-Schmidt in exact
  arithmetic (plain RGS written from its definition);
* Omega Q is orthonormal, W = Q R with R upper triangular with a positive
  diagonal, and T = I_m up to rounding."""
import numpy as np
import pytest

from oracle import rgs, rhqr, sketch
from paper_2405_10923_amd.inputs import synthetic_matrix


def _case(n, m, l, kappa, kind=sketch.SRHT, seed=1):
    W = synthetic_matrix(n, m, kappa, seed=seed)
    sk = sketch.Sketch(kind, n + m, m, l, seed=seed + 7)
    return W, sk


@pytest.mark.parametrize("kind", [sketch.SRHT, sketch.GAUSS])
def test_blas2_rgs_is_rhqr_of_zero_topped_matrix(kind):
    n, m, l = 3000, 12, 60
    W, sk = _case(n, m, l, 3, kind)
    g = rgs.blas2_rgs(W, sk)
    Wb = np.concatenate([np.zeros((m, m)), W], axis=0)
    h = rhqr.rhqr_left(Wb, sk)
    assert np.array_equal(h["U"][:m], np.eye(m))         # head block of U is I exactly
    assert np.all(h["Z"][:m] == 0.0)
    tol = 1e-12
    assert np.max(np.abs(h["U"][m:] - g["Q"])) <= tol * np.max(np.abs(g["Q"]))
    assert np.max(np.abs(-h["R"] - g["R"])) <= tol * np.max(np.abs(g["R"]))
    assert np.max(np.abs(h["T"] - g["T"])) <= tol
    assert np.max(np.abs(h["S"][m:] - g["S"])) <= tol * np.max(np.abs(g["S"]))
    assert np.allclose(h["beta"], 1.0, rtol=0, atol=1e-15)


def test_blas2_rgs_equals_rgs_in_exact_arithmetic():
    n, m, l = 2048, 10, 50
    W, sk = _case(n, m, l, 2)
    g = rgs.blas2_rgs(W, sk)
    r = rgs.rgs(W, sk)
    assert np.max(np.abs(g["Q"] - r["Q"])) <= 1e-12 * np.max(np.abs(r["Q"]))
    assert np.max(np.abs(g["R"] - r["R"])) <= 1e-12 * np.max(np.abs(r["R"]))


@pytest.mark.parametrize("kappa", [2, 10])
def test_blas2_rgs_properties(kappa):
    """Omega Q = S; W = Q R to rounding; R upper triangular with a positive
    diagonal; T unit upper triangular.  Like every Gram-Schmidt process the
    sketched orthogonality and T = I hold to rounding for a well-conditioned
    W and degrade in proportion to cond(W) u otherwise."""
    n, m, l = 4096, 16, 96
    W, sk = _case(n, m, l, kappa)
    g = rgs.blas2_rgs(W, sk)
    Q, R, T, S = g["Q"], g["R"], g["T"], g["S"]
    u = 2.0 ** -53
    tol = max(1e-13, m * 10.0 ** kappa * u)
    assert np.allclose(sk.omega_apply(Q), S, rtol=0, atol=1e-13)
    assert np.linalg.norm(S.T @ S - np.eye(m), 2) <= tol
    assert np.linalg.norm(W - Q @ R) <= 1e-14 * np.linalg.norm(W)
    assert np.array_equal(R, np.triu(R)) and np.all(np.diag(R) > 0)
    assert np.array_equal(T, np.triu(T)) and np.all(np.diag(T) == 1.0)
    assert np.max(np.abs(T - np.eye(m))) <= tol


def test_mutation_missing_resketch_is_caught():
    """A plausible mistake -- keeping the sketch of w_j from before the refresh
    instead of sketching the refreshed vector -- breaks the Omega Q = S pin."""
    n, m, l = 4096, 16, 96
    W, sk = _case(n, m, l, 2)
    Q = np.zeros((n, m))
    S = np.zeros((l, m))
    T = np.eye(m)
    for j in range(m):
        w = W[:, j].copy()
        z = sk.omega_apply(w)
        if j:
            w = w - Q[:, :j] @ (T[:j, :j].T @ (S[:, :j].T @ z))
        Q[:, j], S[:, j] = w / np.linalg.norm(z), z / np.linalg.norm(z)
    assert np.max(np.abs(sk.omega_apply(Q) - S)) > 1e-3
    g = rgs.blas2_rgs(W, sk)
    assert np.max(np.abs(sk.omega_apply(g["Q"]) - g["S"])) <= 1e-13
