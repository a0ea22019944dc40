"""GPU checks of the boundary's contract with a live sketch handle: every
argument error of rhqr_factor / recrhqr_factor / rhqr_sketch returns -i before
anything is launched (the outputs stay untouched), a short workspace returns
RHQR_ERR_WORKSPACE, non-finite input is reported by rhqr_status as -j, the
column scaling equals its definition bit for bit, and the per-kernel profile
window counts the launches of each kernel class."""
import ctypes

import numpy as np
import pytest

from tests.gpu_util import cuda_or_skip, to_gpu, log

pytestmark = pytest.mark.gpu


def _setup(torch, n=3000, m=8, l=64):
    from paper_2405_10923_amd import rhqr
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=3)
    W = to_gpu(np.random.default_rng(0).standard_normal((n, m)))
    b = rhqr.FactorBuffers(sk, torch.float64, m, want_q=True)
    return rhqr, sk, W, b


def test_factor_argument_errors_before_launch():
    torch = cuda_or_skip()
    rhqr, sk, W, b = _setup(torch)
    L = rhqr.lib()
    n, m = W.shape
    P = rhqr._ptr
    Wc = W.clone()
    b.S.fill_(7.0)
    ws = b.ws
    good = [sk.h, 0, n, m, P(W), n, P(b.S), sk.rows_out, P(b.T), m, P(b.R), m, P(b.Q), n, 0,
            P(ws), ws.numel(), rhqr._stream()]

    def call(**kw):
        a = list(good)
        for i, v in kw.items():
            a[int(i[1:]) - 1] = v
        return L.rhqr_factor(*a)

    assert call(a2=5) == -2
    assert call(a3=n + 1) == -3
    assert call(a4=m + 1) == -4
    assert call(a5=None) == -5
    assert call(a6=n - 1) == -6
    assert call(a7=None) == -7
    assert call(a8=sk.rows_out - 1) == -8
    assert call(a9=None) == -9
    assert call(a10=m - 1) == -10
    assert call(a11=None) == -11
    assert call(a12=m - 1) == -12
    assert call(a14=n - 1) == -14
    assert call(a15=7) == -15                       # unknown scaling
    assert call(a15=(33 << 8)) == -15               # panel wider than 32
    assert call(a15=(8 << 8) | (12 << 16)) == -15   # outer not a multiple of the panel
    assert call(a15=(3 << 24)) == -15               # tiles per workgroup not 0, 1, 2 or 4
    assert call(a15=(1 << 28)) == -15               # Alg. 5 needs a block width
    assert call(a15=(1 << 29) | (8 << 8)) == -15    # Alg. 3 takes no schedule bits
    assert call(a15=(1 << 29) | (1 << 28)) == -15
    assert call(a15=(1 << 30)) == -15               # reserved bits
    assert call(a16=None) == -16
    need = L.rhqr_factor_workspace_size(sk.h, 0, m)
    assert call(a17=need - 1) == rhqr.RHQR_ERR_WORKSPACE
    torch.cuda.synchronize()
    assert torch.equal(W, Wc)                        # nothing ran
    assert bool((b.S == 7.0).all())
    assert call() == 0
    torch.cuda.synchronize()
    assert rhqr.status(ws) == 0


def test_recrhqr_and_sketch_argument_errors():
    torch = cuda_or_skip()
    rhqr, sk, W, b = _setup(torch)
    L = rhqr.lib()
    n, m = W.shape
    P = rhqr._ptr
    U = torch.empty_like(W)
    ws = rhqr.workspace(L.recrhqr_workspace_size(sk.h, 0, m), "cuda")
    good = [sk.h, 0, n, m, P(W), n, P(U), n, P(b.S), sk.rows_out, P(b.T), m, P(b.R), m, P(b.Q),
            n, 0, P(ws), ws.numel(), rhqr._stream()]

    def call(**kw):
        a = list(good)
        for i, v in kw.items():
            a[int(i[1:]) - 1] = v
        return L.recrhqr_factor(*a)

    assert call(a2=-1) == -2
    assert call(a5=None) == -5
    assert call(a7=None) == -7
    assert call(a10=3) == -10
    assert call(a17=9) == -17
    assert call(a15=None, a17=1) == -15             # RCHOL needs Q
    assert call(a18=None) == -18
    assert call(a19=16) == rhqr.RHQR_ERR_WORKSPACE
    assert call() == 0
    Y = rhqr.colmajor_empty(sk.rows_out, m, torch.float64, "cuda")
    sws = rhqr.workspace(L.rhqr_sketch_workspace_size(sk.h, m), "cuda")
    assert L.rhqr_sketch(sk.h, 0, n, m, P(W), n, P(Y), sk.rows_out - 1, P(sws), sws.numel(),
                         rhqr._stream()) == -8
    assert L.rhqr_sketch(sk.h, 0, n, m, P(W), n, P(Y), sk.rows_out, P(sws), 8,
                         rhqr._stream()) == rhqr.RHQR_ERR_WORKSPACE
    torch.cuda.synchronize()


@pytest.mark.parametrize("where", ["nan_col3", "inf_col0"])
def test_status_reports_nonfinite_column(where):
    torch = cuda_or_skip()
    rhqr, sk, W, b = _setup(torch)
    j = 3 if where == "nan_col3" else 0
    W[1234, j] = float("nan") if where == "nan_col3" else float("inf")
    for panel in (0, 4):
        Wd = W.clone()
        out = rhqr.factor(sk, Wd, bufs=b, panel=panel)
        assert rhqr.status(out["ws"]) == -(j + 1), (where, panel)
    out = rhqr.recrhqr(sk, W)
    assert rhqr.status(out["ws"]) == -(j + 1)
    # a finite input afterwards resets the status
    Wd = to_gpu(np.random.default_rng(1).standard_normal(tuple(W.shape)))
    out = rhqr.factor(sk, Wd, bufs=b)
    assert rhqr.status(out["ws"]) == 0


@pytest.mark.parametrize("dt", ["float64", "float32", "float16", "bfloat16"])
def test_colscale_definition(dt):
    """d_j = max_i |W_ij| (1 for a zero column); W D^-1 rounded to float32
    and then to the 2-byte type, bit for bit; R D column by column."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    rng = np.random.default_rng(2)
    n, m = 70001, 5
    A = rng.standard_normal((n, m)) * np.array([1e-3, 1.0, 0.0, 3e4, 1.0])
    A[17, 1] = -9.5                                  # the max-abs entry is negative
    W = to_gpu(A)
    dtype = getattr(torch, dt)
    out, d = rhqr.colscale(W, dtype)
    torch.cuda.synchronize()
    dref = np.max(np.abs(A), axis=0)
    dref[dref == 0] = 1.0
    assert np.array_equal(d.cpu().numpy(), dref)
    ref = torch.from_numpy(A / dref)
    if dt != "float64":
        ref = ref.to(torch.float32).to(dtype)
    got = out.cpu().contiguous()
    ref = ref.reshape(got.shape).contiguous()
    if dtype.itemsize == 2:
        gb, rb = got.view(torch.int16), ref.view(torch.int16)
        bad = (gb != rb).nonzero()
        if len(bad):
            i, j = (int(v) for v in bad[0])
            log(f"{dt}: {len(bad)} entries differ, first ({i}, {j}): W/d = {A[i, j] / dref[j]!r} "
                f"gpu {got[i, j].item()!r} ({int(gb[i, j])}) ref {ref[i, j].item()!r} ({int(rb[i, j])})")
        assert len(bad) == 0
    else:
        assert torch.equal(got, ref)
    R = to_gpu(np.triu(rng.standard_normal((m, m))))
    R0 = R.cpu().numpy()
    rhqr.scale_r(R, d)
    assert np.array_equal(R.cpu().numpy(), R0 * dref[None, :])


def test_profile_counts_each_kernel_class():
    torch = cuda_or_skip()
    m = 40
    rhqr, sk, W, b = _setup(torch, n=20000, m=m, l=128)
    rhqr.profile_begin()
    rhqr.factor(sk, W.clone(), bufs=b, panel=8, outer=16, want_q=True)
    torch.cuda.synchronize()
    prof = rhqr.profile_end()
    log(f"profile: {prof}")
    assert prof["tall"][1] == m - 1                  # one refresh pass per column j >= 1
    assert prof["red"][1] == m and prof["fin"][1] == m
    assert prof["presketch"][1] == 1
    assert prof["qtail"][1] == 1
    # panels of 8 in outer panels of 16 over 40 columns: outer updates at 16
    # (16 columns: matrix cores) and 32 (8 columns: vector units), inner
    # updates at 8 and 24 (8 columns: vector units)
    assert prof["panel_mx"][1] == 1 and prof["panel_valu"][1] == 3
    assert all(v[0] > 0 for k, v in prof.items() if v[1])
    rhqr.profile_begin()
    prof2 = rhqr.profile_end()
    assert all(v == (0.0, 0) for v in prof2.values())
