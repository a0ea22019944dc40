"""Pins of the oracle's sketching routine (Sec. 2.3, eq. psi, Alg. 1,
Lemma srht) against dense matrices built independently from scipy's Sylvester
Hadamard matrix, exact integer arithmetic and the embedding property."""
import math

import numpy as np
import pytest
import scipy.linalg

from oracle import sketch, metrics


@pytest.mark.parametrize("N", [1, 2, 8, 64, 1024])
def test_fwht_equals_sylvester_hadamard(N):
    H = scipy.linalg.hadamard(N).astype(np.float64)
    assert np.array_equal(H @ H.T, N * np.eye(N))        # H H^t = N I
    x = np.random.default_rng(N).standard_normal((N, 3))
    assert np.allclose(sketch.fwht(x), H @ x, rtol=0, atol=1e-12 * math.sqrt(N))


def test_fwht_exact_on_integers():
    N = 1 << 12
    x = np.random.default_rng(0).integers(-1, 2, size=N)
    Hi = scipy.linalg.hadamard(N)              # integer matrix
    assert np.array_equal(sketch.fwht(x.astype(np.float64)), (Hi @ x).astype(np.float64))


def _dense_psi(sk):
    """Psi of eq. (psi) as an explicit matrix, Omega = sqrt(N/l) P H D
    restricted to the tail coordinates (H normalised)."""
    n, m, N, l = sk.n, sk.m, sk.N, sk.l
    H = scipy.linalg.hadamard(N).astype(np.float64) / math.sqrt(N)
    D = np.diag(sk.signs)
    Om_full = math.sqrt(N / l) * (H @ D)[sk.rows]           # l x N
    Psi = np.zeros((l + m, n))
    Psi[:m, :m] = np.eye(m)
    Psi[m:, m:] = Om_full[:, m:n]
    return Psi


@pytest.mark.parametrize("n,m,l", [(300, 7, 40), (512, 16, 64), (1000, 3, 30)])
def test_rh_sketch_equals_dense_psi(n, m, l):
    sk = sketch.Sketch(sketch.SRHT, n, m, l, seed=n)
    X = np.random.default_rng(1).standard_normal((n, 5))
    Y = sketch.rh_sketch(X, sk)
    Psi = _dense_psi(sk)
    assert np.allclose(Y, Psi @ X, rtol=0, atol=1e-13 * np.linalg.norm(X))
    assert np.array_equal(Y[:m], X[:m])                    # head block kept


def test_rh_sketch_gaussian_is_head_plus_omega_product():
    n, m, l = 200, 5, 30
    sk = sketch.Sketch(sketch.GAUSS, n, m, l, seed=2)
    X = np.random.default_rng(2).standard_normal((n, 4))
    Y = sketch.rh_sketch(X, sk)
    assert np.array_equal(Y[:m], X[:m])
    Om = sketch.gaussian_omega(2, l, n - m)
    assert np.allclose(Y[m:], Om @ X[m:], rtol=1e-14, atol=1e-14)


def test_srht_integer_input_exact():
    # N/l a power of 4 makes every scale factor a power of two: the sketch of an
    # integer vector is then computed exactly.
    n, m, l = 4096, 8, 64
    sk = sketch.Sketch(sketch.SRHT, n, m, l, seed=5)
    x = np.random.default_rng(5).integers(-3, 4, size=n).astype(np.float64)
    y = sk.omega_apply(x[m:])
    Hi = scipy.linalg.hadamard(n)
    xi = np.zeros(n, dtype=np.int64)
    xi[m:] = x[m:].astype(np.int64) * sk.signs[m:].astype(np.int64)
    exact = (Hi @ xi)[sk.rows] / math.sqrt(l)
    assert np.array_equal(y, exact)


def test_srht_backward_error_within_lemma_bound():
    # Lemma srht: fl(Omega x) = Omega (x + dx), ||dx|| <= gamma_{log2 N + 5} ||x||.
    n, m, l = 2048, 4, 64
    sk = sketch.Sketch(sketch.SRHT, n, m, l, seed=9)
    x = np.random.default_rng(9).standard_normal(n - m)
    y = sk.omega_apply(x)
    Psi = _dense_psi(sk)
    exact = (Psi[m:, m:].astype(np.longdouble) @ x.astype(np.longdouble)).astype(np.float64)
    u = 2.0 ** -53
    k = math.log2(sk.N) + 5
    gam = k * u / (1 - k * u)
    # forward error of the sampled rows is bounded by ||Omega|| ||dx||, ||Omega||_2 <= sqrt(N/l)
    assert np.linalg.norm(y - exact) <= gam * math.sqrt(sk.N / l) * np.linalg.norm(x)


def test_srht_norm_preserved_in_expectation():
    n, m, l = 1024, 4, 32
    x = np.random.default_rng(0).standard_normal(n - m)
    vals = [np.sum(sketch.Sketch(sketch.SRHT, n, m, l, seed=s).omega_apply(x) ** 2)
            for s in range(400)]
    ratio = np.mean(vals) / np.sum(x * x)
    assert abs(ratio - 1.0) < 0.05


@pytest.mark.parametrize("kind", [sketch.SRHT, sketch.GAUSS])
def test_psi_is_an_epsilon_embedding_of_a_range(kind):
    n, m, l = 4096, 16, 64
    W = np.random.default_rng(3).standard_normal((n, m))
    sk = sketch.Sketch(kind, n, m, l, seed=1)
    eps = metrics.embedding_distortion(lambda X: sketch.rh_sketch(X, sk), W)
    assert eps < 0.6


def test_embedding_distortion_pins():
    """epsilon of the embedding definition (Sec. 2.3) on range(W): 0 for the
    identity whatever basis spans the range (so a missing orthonormalisation
    of W fails), |c - 1| for x -> c x, and max(a - 1, 1 - b) for a diagonal map
    with gains a >= b on the coordinate axes spanning the range."""
    rng = np.random.default_rng(0)
    W = np.zeros((50, 2))
    W[0, 0], W[1, 1] = 1.0, 3.0                      # not orthonormal
    assert metrics.embedding_distortion(lambda X: X, W) == pytest.approx(0.0, abs=1e-15)
    G = rng.standard_normal((40, 5))
    assert metrics.embedding_distortion(lambda X: 1.25 * X, G) == pytest.approx(0.25, abs=1e-14)
    D = np.ones(50)
    D[0], D[1] = 1.5, 0.6
    assert metrics.embedding_distortion(lambda X: D[:, None] * X, W) == pytest.approx(0.5, abs=1e-14)
