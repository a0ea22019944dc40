"""Accuracy measures reported in Sec. 8 (figure captions of Figs. perf64,
perf32, perfmixed, reconstruct32): relative Frobenius factorization error,
sketch orthogonality of Psi Q, and condition numbers.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).
"""
import numpy as np


def fact_error(W, Q, R):
    """||W - Q R||_F / ||W||_F."""
    W = np.asarray(W, dtype=np.float64)
    return float(np.linalg.norm(W - Q @ R) / np.linalg.norm(W))


def orth_error(PsiQ):
    """||(Psi Q)^t (Psi Q) - I||_2."""
    G = PsiQ.T @ PsiQ
    return float(np.linalg.norm(G - np.eye(G.shape[0]), 2))


def cond(A):
    s = np.linalg.svd(np.asarray(A, dtype=np.float64), compute_uv=False)
    return float(s[0] / s[-1]) if s[-1] > 0 else float("inf")


def embedding_distortion(sk_apply, W):
    """Largest epsilon with (1-eps)||x|| <= ||Psi x|| <= (1+eps)||x|| on
    range(W) (Definition in Sec. 2.3), via the singular values of Psi Q_W."""
    Qw, _ = np.linalg.qr(np.asarray(W, dtype=np.float64))
    s = np.linalg.svd(sk_apply(Qw), compute_uv=False)
    return float(max(s[0] - 1.0, 1.0 - s[-1]))
