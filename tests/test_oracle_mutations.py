"""Planted mistakes in the oracle (on the CPU) must be caught by the pins:
a flipped pivot sign, a perturbed beta (hence T and the reflector norm), and a
missing re-sketch each break an identity the paper proves."""
import numpy as np
import pytest
import scipy.linalg

from oracle import rhqr, sketch, metrics
from paper_2405_10923_amd.inputs import synthetic_matrix as make_w


def _pins_hold(out, W, sk):
    m = W.shape[1]
    Z = sketch.rh_sketch(W, sk)
    (qr, tau), _ = scipy.linalg.qr(Z, mode="raw")
    Rl = np.triu(qr[:m, :m])
    G = out["S"].T @ out["S"]
    Tw = np.linalg.inv(np.triu(G, 1) + 0.5 * np.diag(np.diag(G)))
    Q = rhqr.thin_q(out["U"], out["T"], m)
    return (np.allclose(out["R"], Rl, atol=1e-12 * np.abs(Rl).max())
            and np.allclose(out["T"], Tw, atol=1e-10)
            and metrics.fact_error(W, Q, out["R"]) < 1e-13
            and metrics.orth_error(sketch.rh_sketch(Q, sk)) < 1e-12)


@pytest.fixture
def problem():
    n, m, l = 400, 8, 32
    return make_w(n, m, 3, seed=21), sketch.Sketch(sketch.SRHT, n, m, l, seed=3)


def test_unmodified_oracle_passes(problem):
    W, sk = problem
    assert _pins_hold(rhqr.rhqr_left(W, sk), W, sk)


def test_flipped_sign_is_caught(problem, monkeypatch):
    W, sk = problem
    orig = rhqr.rh_vector

    def bad(w, y, j, scaling="B"):
        y2 = y.copy()
        y2[j] = -y2[j] if j == 2 else y2[j]
        return orig(w, y2, j, scaling)
    monkeypatch.setattr(rhqr, "rh_vector", bad)
    assert not _pins_hold(rhqr.rhqr_left(W, sk), W, sk)


def test_perturbed_beta_is_caught(problem, monkeypatch):
    W, sk = problem
    orig = rhqr.rh_vector
    calls = {"k": 0}

    def bad(w, y, j, scaling="B"):
        u, s, sg, rho, beta, a, ok = orig(w, y, j, scaling)
        calls["k"] += 1
        return u, s, sg, rho, (beta * 1.0000001 if j == 4 else beta), a, ok
    monkeypatch.setattr(rhqr, "rh_vector", bad)
    assert not _pins_hold(rhqr.rhqr_left(W, sk), W, sk)


def test_missing_resketch_is_caught(problem, monkeypatch):
    W, sk = problem
    real = sketch.rh_sketch
    state = {"calls": 0}

    def stale(X, s):
        # return the sketch of the unrefreshed column for one column's refresh
        state["calls"] += 1
        if state["calls"] == 4:
            return real(W[:, 2], s)
        return real(X, s)
    monkeypatch.setattr(rhqr, "rh_sketch", stale)
    assert not _pins_hold(rhqr.rhqr_left(W, sk), W, sk)
