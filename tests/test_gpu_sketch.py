"""GPU parity of the sketch draw (Sec. 2.3) and of RHSketch (Alg. 1) against
the CPU oracle.  Integer draws (signs, sampled rows) must be bit-exact;
Gaussian entries and sketches agree to rounding."""
import numpy as np
import pytest

from oracle import sketch as osk, philox
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("n,m,l,seed", [(300, 7, 40, 3), (4096, 32, 128, 0),
                                        (3 * 4096 + 777, 24, 96, 11), (1 << 22, 256, 1024, 0)])
def test_srht_draw_bit_exact(n, m, l, seed):
    cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    log(f"srht draw n={n} m={m} l={l} seed={seed}")
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=seed)
    N = osk.next_pow2(n)
    assert sk.N == N
    w_ref = philox.words(seed, philox.STREAM_SIGNS, (N + 63) // 64)
    assert np.array_equal(sk.signs_words(), w_ref)
    assert np.array_equal(sk.rows().astype(np.int64), osk.srht_rows(seed, N, l))


def test_gaussian_draw_matches_oracle():
    cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l, seed = 3000, 10, 64, 5
    sk = rhqr.Sketch(rhqr.GAUSS, n, m, l, seed=seed)
    om = sk.omega()
    ref = osk.gaussian_omega(seed, l, n - m)
    # libm differences in log/cos: a few ulps of the O(1) entries
    assert np.max(np.abs(om - ref)) <= 1e-14 * np.max(np.abs(ref))


@pytest.mark.parametrize("n,m,l,k", [(300, 7, 40, 3), (3 * 4096 + 777, 24, 96, 5),
                                     (5 * 4096, 4, 64, 2),
                                     # 2, 4 and 8 samples per thread, l = TILE
                                     (5000, 6, 600, 2), (3 * 4096 + 5, 10, 1500, 2),
                                     (8192 + 3, 5, 3000, 2), (2 * 4096, 4, 4096, 1)])
def test_srht_sketch_f64(n, m, l, k):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    log(f"srht sketch f64 n={n} m={m} l={l} k={k}")
    X = np.random.default_rng(n).standard_normal((n, k))
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=2)
    Y = to_np(rhqr.sketch(sk, to_gpu(X)))
    ref = osk.rh_sketch(X, osk.Sketch(osk.SRHT, n, m, l, seed=2))
    assert np.array_equal(Y[:m], X[:m])
    for c in range(k):
        assert rel(Y[:, c], ref[:, c]) < 1e-14


def test_srht_sketch_exact_integers():
    cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l = 4 * 4096, 8, 64        # N/l a power of 4: every scale is a power of two
    X = np.random.default_rng(0).integers(-3, 4, size=(n, 2)).astype(np.float64)
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=9)
    Y = to_np(rhqr.sketch(sk, to_gpu(X)))
    ref = osk.rh_sketch(X, osk.Sketch(osk.SRHT, n, m, l, seed=9))
    assert np.array_equal(Y, ref)


@pytest.mark.parametrize("dt", ["float32", "float16", "bfloat16"])
def test_srht_sketch_low_precision(dt):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l, k = 3 * 4096 + 100, 16, 64, 3
    X = np.random.default_rng(1).standard_normal((n, k))
    Xd = to_gpu(X, getattr(torch, dt))
    Xr = to_np(Xd)                      # the rounded input
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=4)
    Y = to_np(rhqr.sketch(sk, Xd))
    ref = osk.rh_sketch(Xr, osk.Sketch(osk.SRHT, n, m, l, seed=4))
    for c in range(k):
        assert rel(Y[:, c], ref[:, c]) < 2e-6      # float32 accumulation


@pytest.mark.parametrize("n,m,l,k", [(9000, 12, 80, 70),
                                     # several 128 x 128 tiles in both directions, ragged
                                     (20000 + 7, 30, 300, 150)])
def test_gauss_sketch_f64(n, m, l, k):
    cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    log(f"gauss sketch f64 n={n} m={m} l={l} k={k}")
    X = np.random.default_rng(3).standard_normal((n, k))
    om = osk.gaussian_omega(6, l, n - m)  # the oracle's draw, handed to the GPU
    sk = rhqr.Sketch(rhqr.GAUSS, n, m, l, seed=6, omega=to_gpu(om))
    Y = to_np(rhqr.sketch(sk, to_gpu(X)))
    ref = np.concatenate([X[:m], om @ X[m:]])
    for c in range(k):
        assert rel(Y[:, c], ref[:, c]) < 1e-13


@pytest.mark.parametrize("dt", ["float32", "float16"])
def test_gauss_sketch_low_precision(dt):
    """Low-precision storage: the product runs in float32 on matrix cores."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l, k = 12000 + 3, 20, 200, 140
    X = np.random.default_rng(5).standard_normal((n, k))
    Xd = to_gpu(X, getattr(torch, dt))
    Xr = to_np(Xd)  # the rounded input
    om = osk.gaussian_omega(7, l, n - m)
    sk = rhqr.Sketch(rhqr.GAUSS, n, m, l, seed=7, omega=to_gpu(om))
    Y = to_np(rhqr.sketch(sk, Xd))
    ref = np.concatenate([Xr[:m], om @ Xr[m:]])
    # float32 products of n - m terms: well inside the storage type's tolerance
    assert rel(Y, ref) < (1e-5 if dt == "float32" else 1e-4)


def test_sketch_large_column_sampled():
    """c3 shape (2^22 rows): sampled columns against the oracle."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    from paper_2405_10923_amd.inputs import synthetic_matrix_torch
    n, m, l = 1 << 22, 256, 1024
    log("sketch 2^22 x 4 sampled")
    W = synthetic_matrix_torch(n, 4, 2, seed=0)
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=0)
    Y = to_np(rhqr.sketch(sk, W))
    Wn = to_np(W)
    ref = osk.rh_sketch(Wn, osk.Sketch(osk.SRHT, n, m, l, seed=0))
    for c in range(4):
        assert rel(Y[:, c], ref[:, c]) < 1e-13
