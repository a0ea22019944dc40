"""GPU parity of left-looking trimRHQR (Alg. 12 with trimRHVector, Alg. 10)
against the oracle: element-wise U, S = Omega U, T, T~, R and the thin Q on
well-conditioned inputs (several tiles with a ragged tail, both scalings,
sketches with fewer rows than columns), bounds for float32 and for an
ill-conditioned float64 input, breakdown on a zero column."""
import numpy as np
import pytest

from oracle import trim as otrim
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu


def _run(W, l, dtype="float64", scaling=0, seed=4):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m = W.shape
    sk = rhqr.Sketch(rhqr.SRHT, n, 0, l, seed=seed)
    Wd = to_gpu(W, getattr(torch, dtype))
    Win = to_np(Wd)
    out = rhqr.trim(sk, Wd, scaling=scaling)
    torch.cuda.synchronize()
    info = rhqr.status(out["ws"])
    g = {k: to_np(out[k]) for k in ("U", "S", "T", "Tt", "R", "Q")}
    return g, Win, otrim.FullSketch(n, l, seed=seed), info


@pytest.mark.parametrize("n,m,l,scaling", [
    (3000, 10, 40, 0),
    (3 * 4096 + 777, 24, 96, 0),
    (3 * 4096 + 777, 24, 96, 1),
    (2 * 4096 + 5, 48, 32, 0),      # fewer sketch rows than columns
    (5000, 64, 64, 0),
])
def test_trim_elementwise(n, m, l, scaling):
    log(f"trim n={n} m={m} l={l} scaling={scaling}")
    W = synthetic_matrix(n, m, 2, seed=3)
    g, _, om, info = _run(W, l, scaling=scaling)
    assert info == 0
    ref = otrim.trim_rhqr_left(W, om, "B" if scaling == 0 else "A")
    for k in ("U", "S", "R"):
        assert rel(g[k], ref[k]) < 1e-12, k
    assert np.max(np.abs(g["T"] - ref["T"])) <= 1e-12 * np.max(np.abs(ref["T"]))
    assert np.max(np.abs(g["Tt"] - ref["Tt"])) <= 1e-12 * np.max(np.abs(ref["Tt"]))
    Qref = otrim.trim_thin_q(ref["U"], ref["T"], ref["S"], ref["E"], m)
    assert rel(g["Q"], Qref) < 1e-12


@pytest.mark.parametrize("dt,tol,kappa", [("float64", 1e-12, 10), ("float32", 1e-5, 5)])
def test_trim_bounds(dt, tol, kappa):
    n, m, l = 3 * 4096 + 99, 32, 128
    W = synthetic_matrix(n, m, kappa, seed=5)
    g, Win, om, info = _run(W, l, dtype=dt)
    assert info == 0
    ef = np.linalg.norm(Win - g["Q"] @ g["R"]) / np.linalg.norm(Win)
    log(f"trim {dt} cond 1e{kappa}: e_fact {ef:.2e}")
    assert ef < tol


def test_trim_zero_column_breakdown():
    n, m, l = 3000, 8, 40
    W = synthetic_matrix(n, m, 1, seed=6)
    W[:, 3] = 0.0
    g, _, om, info = _run(W, l)
    assert info == 4
