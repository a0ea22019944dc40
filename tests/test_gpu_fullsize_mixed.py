"""GPU parity of the low-precision storage types at full size, and of the
tall pass with two transform tiles per workgroup.

* 2^22 x 256, cond 1e14, SRHT l = 1024 (the mixed-precision workload), for
  float32, float16 and bfloat16 with the blocked schedules the benchmark
  times; W is scaled to unit max-norm columns and rounded by rhqr_colscale.
* n = 3 * 2^20 + 1234 (between 2^21 and 2^22, so each tall workgroup covers
  two 4096-row tiles and the last one is ragged), m = 64, l = 512, cond 1e8,
  float64 / float32 / float16, blocked and column schedules.

The oracle cannot factor these sizes in seconds, so every check evaluates
the oracle's Psi (its sign and row draw) on the outputs, with the torch
helper pinned against the oracle on the CPU, plus float64 torch products:

* e_fact = ||W~ - Q R|| / ||W~|| (W~ the stored input) and, with R scaled
  back by the column scales, ||W - Q R D|| / ||W|| against the float64 W;
* e_orth = ||(Psi Q)^t Psi Q - I||_2 with Psi Q formed from the returned Q;
* S = Psi U column by column, U as stored: rounding U to the storage type
  (twice: the raw column, then u = w~/alpha) moves each column by at most
  2u of its norm, and the float32 tile transform of the sketch adds the SRHT
  backward error gamma_{log2 N + 5} of Sec. 4, each magnified by at most
  (1+eps)/(1-eps) <= 3 for these embeddings;
* Psi W~ = (I - S T S^t) [R; 0] column by column (the compact form of
  Prop. 3.2 under Psi), to the workload's tolerance.

Tolerances: float64 1e-12, float32 1e-5, float16 / bfloat16 1e-2."""
import math

import numpy as np
import pytest

from oracle import sketch as osk
from tests.gpu_util import cuda_or_skip, psi_apply_torch, cond_gram, orth_err, log

pytestmark = pytest.mark.gpu

TOL = {"float64": 1e-12, "float32": 1e-5, "float16": 1e-2, "bfloat16": 1e-2}
UNIT = {"float64": 2.0 ** -53, "float32": 2.0 ** -24, "float16": 2.0 ** -11, "bfloat16": 2.0 ** -8}
SCHED = {"float64": (8, 32), "float32": (8, 32), "float16": (16, 0), "bfloat16": (16, 0)}

_OSK = {}


def _osketch(n, m, l, seed=0):
    key = (n, m, l, seed)
    if key not in _OSK:
        _OSK.clear()
        _OSK[key] = osk.Sketch(osk.SRHT, n, m, l, seed=seed)
    return _OSK[key]


def _sketch_tol(dt, N):
    u32 = UNIT["float64"] if dt == "float64" else UNIT["float32"]
    # both sides transform: the library in its tile pass, the check in torch
    return 3.0 * (2.0 * UNIT[dt] + 2.0 * (math.log2(N) + 5) * u32) + 1e-14


def check_factorization(torch, rhqr, W64, Wst, d, out, osketch, dt, what):
    """The checks listed in the module docstring; returns the metrics."""
    m = W64.shape[1]
    tol = TOL[dt]
    assert rhqr.status(out["ws"]) == 0, what
    U, S, T, R, Q = out["U"], out["S"], out["T"], out["R"], out["Q"]
    Wt = Wst.to(torch.float64)
    Qd = Q.to(torch.float64)
    ef = float(torch.linalg.norm(Wt - Qd @ R) / torch.linalg.norm(Wt))
    if d is not None:
        R64 = rhqr.scale_r(R.clone().t().contiguous().t(), d)
        ef64 = float(torch.linalg.norm(W64 - Qd @ R64) / torch.linalg.norm(W64))
    else:
        ef64 = ef
    PQ = psi_apply_torch(osketch, Qd)
    eo = orth_err(PQ)
    cq = cond_gram(Qd)
    del Qd
    PU = psi_apply_torch(osketch, U)
    s_err = float(((PU - S).norm(dim=0) / S.norm(dim=0)).max())
    del PU
    Z = psi_apply_torch(osketch, Wt)
    Rp = torch.zeros_like(Z)
    Rp[:m] = R
    CZ = Rp - S @ (T @ (S.t() @ Rp))
    z_err = float(((CZ - Z).norm(dim=0) / Z.norm(dim=0)).max())
    del Z, CZ, Rp, Wt
    stol = _sketch_tol(dt, osketch.N)
    log(f"{what}: e_fact {ef:.2e} (vs f64 W {ef64:.2e}) e_orth {eo:.2e} cond(Q) {cq:.4f} "
        f"|S - Psi U| {s_err:.2e} (bound {stol:.1e}) |Psi W - (I - STS^t)R| {z_err:.2e}")
    assert ef <= tol and ef64 <= tol, (what, ef, ef64)
    assert eo <= tol, (what, eo)
    assert s_err <= stol, (what, s_err)
    assert z_err <= tol, (what, z_err)
    return {"e_fact": ef, "e_fact64": ef64, "e_orth": eo, "cond_Q": cq}


def _run(torch, rhqr, n, m, l, kappa, dt, panel, outer, what):
    from paper_2405_10923_amd.inputs import synthetic_matrix_torch
    W64 = synthetic_matrix_torch(n, m, kappa, seed=0, device="cuda")
    dtype = getattr(torch, dt)
    if dt == "float64":
        Wst, d = W64, None
    else:
        Wst, d = rhqr.colscale(W64, dtype)
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=0)
    Wd = Wst.clone()
    out = rhqr.factor(sk, Wd, want_q=True, panel=panel, outer=outer)
    torch.cuda.synchronize()
    res = check_factorization(torch, rhqr, W64, Wst, d, out, _osketch(n, m, l), dt, what)
    del out, Wd, W64, Wst
    torch.cuda.empty_cache()
    return res


@pytest.mark.parametrize("dt", ["float32", "float16", "bfloat16"])
def test_c3_mixed_fullsize(dt):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l = 1 << 22, 256, 1024
    panel, outer = SCHED[dt]
    log(f"c3 {dt} panel={panel} outer={outer}: W {n} x {m} cond 1e14, SRHT l={l}")
    _run(torch, rhqr, n, m, l, 14, dt, panel, outer, f"c3 {dt}")


@pytest.mark.parametrize("dt,panel,outer", [("float64", 8, 32), ("float64", 0, 0),
                                            ("float32", 8, 32), ("float32", 0, 0),
                                            ("float16", 16, 0)])
def test_two_tiles_per_workgroup(dt, panel, outer):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l = 3 * (1 << 20) + 1234, 64, 512
    log(f"tpw2 {dt} panel={panel} outer={outer}: W {n} x {m} cond 1e8, SRHT l={l}")
    _run(torch, rhqr, n, m, l, 8, dt, panel, outer, f"tpw2 {dt} {panel}/{outer}")
