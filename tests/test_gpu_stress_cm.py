"""The paper's stress input C_m (Sec. 8): n = 50000, C_ij = f((i-1)/(n-1),
(j-1)/(m-1)) with f(x, mu) = sin(10(mu+x)) / (cos(100(mu-x)) + 1.1), which is
numerically singular in float64 from about its 500th column.  m = 600, SRHT
l = 4096 (N = 65536).

Checked on the GPU next to the oracle's own float64 run:
* RHQR (Sec. 4 and Sec. 8, Figs. perf64 and perf32): the sketch Psi Q of the
  basis stays numerically orthogonal and the factorization accurate past the
  point where W becomes singular, in float64 and float32, independently of
  cond(W); Q is then as well conditioned as the embedding allows (below 2 at
  the paper's sampling sizes; 2.07 for the oracle with this draw).  Past the
  numerical rank the computed basis is set by rounding, so the GPU's cond(Q)
  is compared with the oracle's to 10 %, not digit for digit.
* recRHQR and randomized Cholesky QR (Sec. 8, Fig. reconstruct32): both
  backward stable (e_fact at rounding level); in float64 recRHQR's cond(Q) is
  below the paper's bound of 5.  The values in float32, where C_600 is far
  beyond singular, are logged for the record.
The oracle runs in float64 on the host once per module."""
import numpy as np
import pytest

from oracle import sketch as osk, rhqr as orq, metrics
from paper_2405_10923_amd.inputs import cm_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, log

pytestmark = pytest.mark.gpu

N_ROWS, M, L = 50000, 600, 4096


@pytest.fixture(scope="module")
def cm():
    W = cm_matrix(N_ROWS, M)
    sk = osk.Sketch(osk.SRHT, N_ROWS, M, L, seed=0)
    ref = orq.rhqr_left(W, sk)
    Q = orq.thin_q(ref["U"], ref["T"], M)
    rec = orq.rec_rhqr(W, sk, "M")
    rch = orq.rec_rhqr(W, sk, "R")
    out = {"W": W, "sk": sk}
    for name, (Qx, Rx) in (("rhqr", (Q, ref["R"])), ("rec", (rec["Q"], rec["R"])),
                           ("rchol", (rch["Q"], rch["R"]))):
        out[name] = {"e_fact": metrics.fact_error(W, Qx, Rx),
                     "e_orth": metrics.orth_error(osk.rh_sketch(Qx, sk)),
                     "cond_Q": metrics.cond(Qx)}
    log(f"C_{M} oracle: {[(k, out[k]) for k in ('rhqr', 'rec', 'rchol')]}")
    return out


def _metrics(W, Q, R, sk):
    Qn, Rn = to_np(Q), to_np(R)
    return {"e_fact": metrics.fact_error(W, Qn, Rn),
            "e_orth": metrics.orth_error(osk.rh_sketch(Qn, sk)), "cond_Q": metrics.cond(Qn)}


def _stored(torch, rhqr, W, dt):
    """W in the storage type: float64 as is, otherwise unit max-norm columns
    rounded by rhqr_colscale; returns (stored W on the GPU, its float64 copy
    on the host, column scales)."""
    W64 = to_gpu(W)
    if dt == "float64":
        return W64, W, None
    Ws, d = rhqr.colscale(W64, getattr(torch, dt))
    return Ws, to_np(Ws), d


@pytest.mark.parametrize("dt,panel,outer", [("float64", 8, 32), ("float64", 0, 0),
                                            ("float32", 8, 32)])
def test_cm_rhqr(cm, dt, panel, outer):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    Ws, Wn, d = _stored(torch, rhqr, cm["W"], dt)
    sk = rhqr.Sketch(rhqr.SRHT, N_ROWS, M, L, seed=0)
    out = rhqr.factor(sk, Ws.clone(), want_q=True, panel=panel, outer=outer)
    torch.cuda.synchronize()
    info = rhqr.status(out["ws"])
    g = _metrics(Wn, out["Q"], out["R"], cm["sk"])
    o = cm["rhqr"]
    log(f"C_{M} RHQR {dt} {panel}/{outer}: gpu {g} status {info}; oracle {o}")
    tol = 1e-12 if dt == "float64" else 1e-5
    assert g["e_fact"] <= tol and g["e_orth"] <= tol
    assert o["e_fact"] <= 1e-12 and o["e_orth"] <= 1e-12
    assert g["cond_Q"] < 2.5
    assert abs(g["cond_Q"] - o["cond_Q"]) <= 0.1 * o["cond_Q"]


@pytest.mark.parametrize("dt", ["float64", "float32"])
def test_cm_recrhqr_and_rchol(cm, dt):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    Ws, Wn, d = _stored(torch, rhqr, cm["W"], dt)
    sk = rhqr.Sketch(rhqr.SRHT, N_ROWS, M, L, seed=0)
    rec = rhqr.recrhqr(sk, Ws, mode=rhqr.REC_M, want_q=True)
    rch = rhqr.recrhqr(sk, Ws, mode=rhqr.REC_RCHOL, want_q=True)
    torch.cuda.synchronize()
    gr = _metrics(Wn, rec["Q"], rec["R"], cm["sk"])
    gc = _metrics(Wn, rch["Q"], rch["R"], cm["sk"])
    log(f"C_{M} {dt}: recRHQR gpu {gr}, RCholQR gpu {gc}; oracle rec {cm['rec']}, "
        f"rchol {cm['rchol']}")
    tol = 1e-12 if dt == "float64" else 1e-5
    assert gr["e_fact"] <= tol and gc["e_fact"] <= tol
    if dt == "float64":
        assert gr["cond_Q"] < 5.0
