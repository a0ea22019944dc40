"""GPU parity of block RHQR as Alg. 5 writes it (rhqr_factor opts bit 28:
every earlier block applied to the current block after a fresh sketch of it,
then Alg. 4 inside the block) against the oracle's Alg. 5: element-wise on
well-conditioned inputs for several block widths, sketches and ragged
shapes; through the factorization error and sketched orthogonality on an
ill-conditioned input and in low precision.  The two GPU schedules (Alg. 5
and the panel-product schedule) compute the same factorization."""
import numpy as np
import pytest

from oracle import sketch as osk, rhqr as orq, metrics
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu

ALG5 = 1 << 28


def _factor(W, n, m, l, b, kind="srht", dtype="float64", seed=0):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    okind = osk.SRHT if kind == "srht" else osk.GAUSS
    osketch = osk.Sketch(okind, n, m, l, seed=seed + 5)
    om = to_gpu(osketch.omega) if kind == "gauss" else None
    sk = rhqr.Sketch(rhqr.SRHT if kind == "srht" else rhqr.GAUSS, n, m, l, seed=seed + 5,
                     omega=om)
    Wd = to_gpu(W, getattr(torch, dtype))
    Win = to_np(Wd)
    bufs = rhqr.FactorBuffers(sk, Wd.dtype, m, want_q=True)
    P = rhqr._ptr
    rc = rhqr.lib().rhqr_factor(sk.h, rhqr.dtype_code(Wd.dtype), n, m, P(Wd), rhqr._ld(Wd),
                                P(bufs.S), rhqr._ld(bufs.S), P(bufs.T), rhqr._ld(bufs.T),
                                P(bufs.R), rhqr._ld(bufs.R), P(bufs.Q), rhqr._ld(bufs.Q),
                                ALG5 | (b << 8), P(bufs.ws), bufs.ws.numel(), rhqr._stream())
    assert rc == 0
    torch.cuda.synchronize()
    assert rhqr.status(bufs.ws) == 0
    g = {"U": to_np(Wd), "S": to_np(bufs.S), "T": to_np(bufs.T), "R": to_np(bufs.R),
         "Q": to_np(bufs.Q)}
    return g, osketch, Win


@pytest.mark.parametrize("n,m,l,b,kind", [
    (3000, 12, 64, 4, "srht"),
    (3 * 4096 + 555, 40, 160, 8, "srht"),
    (3 * 4096 + 555, 40, 160, 16, "srht"),
    (2 * 4096 + 3, 37, 150, 32, "srht"),
    (2 * 4096 + 3, 20, 80, 1, "srht"),
    (2 * 4096 + 21, 24, 96, 8, "gauss"),
])
def test_alg5_elementwise(n, m, l, b, kind):
    log(f"alg5 n={n} m={m} l={l} b={b} {kind}")
    W = synthetic_matrix(n, m, 2, seed=1)
    g, sk, _ = _factor(W, n, m, l, b, kind)
    ref = orq.block_rhqr(W, sk, b)
    for k in ("U", "S", "R"):
        assert rel(g[k], ref[k]) < 1e-12, k
    # each block's T is the diagonal block of the library's T
    for i, Tb in enumerate(ref["Ts"]):
        J = i * b
        kb = Tb.shape[0]
        assert rel(g["T"][J:J + kb, J:J + kb], Tb) < 1e-12, i
    # and the full T equals Alg. 4's (same reflectors)
    ref4 = orq.rhqr_left(W, sk)
    assert rel(g["T"], ref4["T"]) < 1e-12
    assert rel(g["Q"], orq.thin_q(ref4["U"], ref4["T"], m)) < 1e-12


@pytest.mark.parametrize("dt,tol,kappa", [("float64", 1e-12, 10), ("float32", 1e-5, 6),
                                          ("float16", 1e-2, 3), ("bfloat16", 1e-2, 3)])
def test_alg5_bounds(dt, tol, kappa):
    n, m, l, b = 3 * 4096 + 99, 32, 128, 8
    W = synthetic_matrix(n, m, kappa, seed=2)
    g, sk, Win = _factor(W, n, m, l, b, dtype=dt)
    ef = metrics.fact_error(Win, g["Q"], g["R"])
    eo = metrics.orth_error(osk.rh_sketch(g["Q"], sk))
    log(f"alg5 {dt} cond 1e{kappa}: e_fact {ef:.2e} e_orth {eo:.2e}")
    assert ef < tol and eo < tol
