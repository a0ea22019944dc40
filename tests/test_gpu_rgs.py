"""GPU parity of BLAS2-RGS (Alg. 9, Sec. 6) against the oracle's Alg. 9:
element-wise on well-conditioned inputs (Q, R, T, S = Omega Q), over the
column and blocked schedules, the SRHT and the Gaussian sketch and several
tiles with a ragged tail; through the factorization error and the sketched
orthogonality for the low-precision storage types."""
import numpy as np
import pytest

from oracle import sketch as osk, rgs as orgs, metrics
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu


def _run(n, m, l, kappa, kind="srht", dtype="float64", panel=0, outer=0, seed=0):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    W = synthetic_matrix(n, m, kappa, seed=seed)
    okind = osk.SRHT if kind == "srht" else osk.GAUSS
    osketch = osk.Sketch(okind, n + m, m, l, seed=seed + 11)
    om = to_gpu(osketch.omega) if kind == "gauss" else None
    sk = rhqr.Sketch(rhqr.SRHT if kind == "srht" else rhqr.GAUSS, n + m, m, l, seed=seed + 11,
                     omega=om)
    Wd = to_gpu(W, getattr(torch, dtype))
    out = rhqr.rgs(sk, Wd, panel=panel, outer=outer)
    torch.cuda.synchronize()
    assert rhqr.status(out["ws"]) == 0
    g = {k: to_np(out[k]) for k in ("Q", "Qfull", "S", "T", "R")}
    return W, to_np(Wd), g, osketch


@pytest.mark.parametrize("n,m,l,panel,outer,kind", [
    (3000, 9, 64, 0, 0, "srht"),
    (3 * 4096 + 321, 24, 128, 0, 0, "srht"),
    (3 * 4096 + 321, 24, 128, 8, 0, "srht"),
    (2 * 4096 + 5, 40, 160, 4, 16, "srht"),
    (2 * 4096 + 77, 16, 64, 0, 0, "gauss"),
])
def test_blas2_rgs_elementwise(n, m, l, panel, outer, kind):
    log(f"rgs n={n} m={m} l={l} panel={panel}/{outer} {kind}")
    W, Win, g, sk = _run(n, m, l, 2, kind=kind, panel=panel, outer=outer)
    ref = orgs.blas2_rgs(W, sk)
    assert np.array_equal(g["Qfull"][:m], np.eye(m))
    assert rel(g["Q"], ref["Q"]) < 1e-12
    assert rel(g["R"], ref["R"]) < 1e-12
    assert np.max(np.abs(g["T"] - ref["T"])) < 1e-12
    assert np.array_equal(g["S"][:m], np.eye(m))
    assert rel(g["S"][m:], ref["S"]) < 1e-12
    assert np.all(np.diag(g["R"]) > 0)


@pytest.mark.parametrize("dt,tol", [("float32", 1e-5), ("float16", 1e-2), ("bfloat16", 1e-2)])
def test_blas2_rgs_low_precision(dt, tol):
    """A Gram-Schmidt process loses sketched orthogonality in proportion to
    cond(W) u (Sec. 6 compares it with RGS, whose bound has that form), so
    the low-precision check uses a well-conditioned W (singular values all
    1): what remains is the rounding of Q to the storage type."""
    n, m, l = 3 * 4096 + 99, 24, 128
    W, Win, g, sk = _run(n, m, l, 0, dtype=dt, panel=8)
    ef = metrics.fact_error(Win, g["Q"], g["R"])
    eo = metrics.orth_error(sk.omega_apply(g["Q"]))
    log(f"rgs {dt}: e_fact {ef:.2e} e_orth {eo:.2e}")
    assert ef < tol and eo < tol
