"""GPU parity of recRHQR (Alg. 6) and its randomized-Cholesky-QR mode
against the CPU oracle: element-wise on well-conditioned inputs, through the
factorization error and the sketch orthogonality on ill-conditioned ones."""
import numpy as np
import pytest

from oracle import sketch as osk, rhqr as orq, metrics
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu


def _rec(n, m, l, kappa, mode, dtype="float64", seed=0, kind=0):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    W = synthetic_matrix(n, m, kappa, seed=seed)
    Wd = to_gpu(W, getattr(torch, dtype))
    okind = osk.SRHT if kind == rhqr.SRHT else osk.GAUSS
    osketch = osk.Sketch(okind, n, m, l, seed=seed + 3)
    # Gaussian: the oracle's Omega (its own Philox draw) is handed to the GPU
    om = to_gpu(osketch.omega) if kind == rhqr.GAUSS else None
    sk = rhqr.Sketch(kind, n, m, l, seed=seed + 3, omega=om)
    out = rhqr.recrhqr(sk, Wd, mode=mode, want_q=True)
    torch.cuda.synchronize()
    g = {k: (to_np(v) if v is not None else None) for k, v in out.items() if k != "ws"}
    return W, to_np(Wd), g, osketch


# m = 128 fills the matrix-core substitution's eight column blocks; m = 136
# takes the blocked substitution (m > 128)
@pytest.mark.parametrize("n,m,l", [(300, 7, 40), (3 * 4096 + 777, 24, 96), (2 * 4096 + 5, 70, 200),
                                   (2 * 4096 + 9, 128, 300), (4096 + 21, 136, 300)])
def test_rec_m_elementwise(n, m, l):
    log(f"recrhqr M n={n} m={m} l={l}")
    W, Win, g, sk = _rec(n, m, l, 2, 0)
    ref = orq.rec_rhqr(W, sk, "M")
    for k in ("S", "T", "R", "U", "Q"):
        assert rel(g[k], ref[k]) < 1e-12, k


def test_rec_rchol_elementwise():
    n, m, l = 3 * 4096 + 100, 20, 80
    W, Win, g, sk = _rec(n, m, l, 2, 1)
    ref = orq.rec_rhqr(W, sk, "R")
    assert rel(g["R"], ref["R"]) < 1e-12
    assert rel(g["Q"], ref["Q"]) < 1e-12


def test_rec_gauss():
    n, m, l = 2 * 4096 + 17, 16, 64
    W, Win, g, sk = _rec(n, m, l, 2, 0, kind=1)
    ref = orq.rec_rhqr(W, sk, "M")
    for k in ("S", "T", "R", "U", "Q"):
        assert rel(g[k], ref[k]) < 1e-12, k


def test_rec_ill_conditioned_bounds():
    n, m, l = 4096, 32, 128
    W, Win, g, sk = _rec(n, m, l, 8, 0)
    ref = orq.rec_rhqr(W, sk, "M")
    ef = metrics.fact_error(W, g["Q"], g["R"])
    eo = metrics.orth_error(osk.rh_sketch(g["Q"], sk))
    ef_o = metrics.fact_error(W, ref["Q"], ref["R"])
    eo_o = metrics.orth_error(osk.rh_sketch(ref["Q"], sk))
    log(f"rec cond 1e8: e_fact {ef:.2e} ({ef_o:.2e})  e_orth {eo:.2e} ({eo_o:.2e})")
    assert ef < 1e-12
    assert abs(ef - ef_o) < 1e-12
    # recRHQR's sketch orthogonality degrades in proportion to cond(W) u (Sec. 8,
    # Fig. reconstruct32); the loss is rounding-dependent, so the GPU value
    # must be of the oracle's order of magnitude and below cond(W) m u.
    assert eo < 1e8 * m * 2.0 ** -53
    assert 0.1 < eo / eo_o < 10.0


@pytest.mark.parametrize("dt,tol", [("float32", 1e-5), ("float16", 1e-2), ("bfloat16", 1e-2)])
def test_rec_low_precision(dt, tol):
    n, m, l = 3 * 4096 + 77, 24, 96
    W, Win, g, sk = _rec(n, m, l, 2, 0, dtype=dt)
    ef = metrics.fact_error(Win, g["Q"], g["R"])
    eo = metrics.orth_error(osk.rh_sketch(g["Q"], sk))
    log(f"rec {dt}: e_fact {ef:.2e} e_orth {eo:.2e}")
    assert ef < tol and eo < tol


@pytest.mark.parametrize("mode", [0, 1])
def test_rec_psi_identity_fallback_elementwise(mode):
    """l + 2m > 2048: the sketch-space QR runs the column engine with Psi = I
    instead of the panel kernels (the path C_m with m = 600 takes)."""
    n, m, l = 8192, 64, 2000
    log(f"recrhqr fallback mode={mode} n={n} m={m} l={l} (l + 2m = {l + 2 * m})")
    W, Win, g, sk = _rec(n, m, l, 2, mode)
    ref = orq.rec_rhqr(W, sk, "M" if mode == 0 else "R")
    keys = ("S", "T", "R", "U", "Q") if mode == 0 else ("S", "T", "R", "Q")
    for k in keys:
        assert rel(g[k], ref[k]) < 1e-12, k
