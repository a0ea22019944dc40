"""GPU parity of the batched left-looking RHQR (rhqr_batch_*).

Every problem of a batch is compared (a) bitwise with the single-problem
rhqr_factor (column schedule) on the same input, since both run the same
device code in the same reduction order, and (b) with the CPU oracle, element
by element for well-conditioned inputs and through the factorization error and
sketch orthogonality bounds otherwise.  The hipGraph form is replayed several
times with other GPU work in between and every replay is checked against the
eager result."""
import numpy as np
import pytest

from oracle import sketch as osk, rhqr as orq, metrics
from paper_2405_10923_amd.inputs import synthetic_matrix
from tests.gpu_util import cuda_or_skip, to_gpu, to_np, rel, log

pytestmark = pytest.mark.gpu

# (n, m, l, seed): ragged and power-of-two n, several tiles and a partial tile,
# m from 7 to 70, so problems drop out of the batch at different columns
SHAPES = [(5000, 12, 48, 1), (4096, 32, 128, 2), (3 * 4096 + 777, 24, 96, 3), (300, 7, 40, 4),
          (2 * 8192 + 1, 40, 160, 5), (16384, 16, 64, 6), (2 * 4096 + 5, 70, 200, 7)]


def _sched(panel):
    """(panel, outer) of a schedule parameter: a panel width or a pair."""
    return panel if isinstance(panel, tuple) else (panel, 0)


def _inputs(torch, dt, kappa=3.0, shapes=SHAPES):
    from paper_2405_10923_amd import rhqr
    probs = []
    for n, m, l, seed in shapes:
        W = synthetic_matrix(n, m, kappa, seed=seed)
        probs.append((W, rhqr.Sketch(rhqr.SRHT, n, m, l, seed=seed + 100), (n, m, l, seed)))
    return probs


@pytest.mark.parametrize("panel", [0, 16, (8, 32), (5, 15)])
@pytest.mark.parametrize("dt", ["float64", "float32", "float16", "bfloat16"])
def test_batch_bitwise_equals_single(dt, panel):
    """Same schedule, same device code, same choice of units for every panel
    (matrix cores for panels wider than 8 with aligned columns, vector units
    otherwise): bitwise equal in every storage type."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    tdt = getattr(torch, dt)
    probs = _inputs(torch, tdt)
    log(f"batch {dt} panel={panel}: {len(probs)} problems")
    batch_in = [(sk, to_gpu(W, tdt)) for W, sk, _ in probs]
    pn, outer = _sched(panel)
    b = rhqr.Batch(batch_in, panel=pn, outer=outer)
    outs = b.factor()
    torch.cuda.synchronize()
    assert b.status() == [0] * len(probs)
    for (W, sk, shp), o in zip(probs, outs):
        log(f"  single {shp}")
        Wd = to_gpu(W, tdt)
        ref = rhqr.factor(sk, Wd, panel=pn, outer=outer)
        torch.cuda.synchronize()
        for k in ("U", "S", "T", "R"):
            assert torch.equal(o[k], ref[k]), (shp, k)
    b.close()


def test_batch_large_sketches_bitwise():
    """Problems whose sketches take 2 and 8 samples per thread in the
    pre-sketch (l = 600 and 3000): the batch equals the single-problem
    factorization bitwise."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    probs = _inputs(torch, torch.float64, shapes=[(5000, 20, 600, 21), (8192 + 3, 12, 3000, 22)])
    b = rhqr.Batch([(sk, to_gpu(W)) for W, sk, _ in probs], panel=16)
    outs = b.factor()
    torch.cuda.synchronize()
    assert b.status() == [0] * len(probs)
    for (W, sk, shp), o in zip(probs, outs):
        log(f"  single {shp}")
        ref = rhqr.factor(sk, to_gpu(W), panel=16)
        torch.cuda.synchronize()
        for k in ("U", "S", "T", "R"):
            assert torch.equal(o[k], ref[k]), (shp, k)
    b.close()


@pytest.mark.parametrize("panel", [0, 16, (8, 32)])
def test_batch_f64_matches_oracle(panel):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    probs = _inputs(torch, torch.float64, kappa=2.0)
    pn, outer = _sched(panel)
    b = rhqr.Batch([(sk, to_gpu(W)) for W, sk, _ in probs], panel=pn, outer=outer)
    outs = b.factor()
    torch.cuda.synchronize()
    for (W, sk, (n, m, l, seed)), o in zip(probs, outs):
        log(f"  oracle {n} {m} {l}")
        ref = orq.rhqr_left(W, osk.Sketch(osk.SRHT, n, m, l, seed=seed + 100))
        for k in ("U", "S", "T", "R"):
            assert rel(to_np(o[k]), ref[k]) < 1e-12, (n, m, l, k)
    b.close()


@pytest.mark.parametrize("panel", [0, 16, (8, 32)])
def test_batch_graph_replays_match_eager(panel):
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    probs = _inputs(torch, torch.float32)
    src = [to_gpu(W, torch.float32) for W, _, _ in probs]
    work = [s.clone() for s in src]
    pn, outer = _sched(panel)
    b = rhqr.Batch([(sk, w) for (_, sk, _), w in zip(probs, work)], panel=pn, outer=outer)
    eager = [{k: v.clone() for k, v in o.items()} for o in b.factor(graph=False)]
    torch.cuda.synchronize()
    for rep in range(3):
        for s, w in zip(src, work):
            w.copy_(s)  # the batch overwrites W with U: restore the input
        junk = torch.randn(1 << 20, device="cuda").sum()  # unrelated eager work
        outs = b.factor(graph=True)
        torch.cuda.synchronize()
        log(f"  replay {rep} (eager work {float(junk):.3f})")
        for e, o in zip(eager, outs):
            for k in ("U", "S", "T", "R"):
                assert torch.equal(e[k], o[k]), (rep, k)
    b.close()


def test_batch_rank_deficient_problem_reported():
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    n, m, l = 5000, 10, 40
    W0 = synthetic_matrix(n, m, 2.0, seed=11)
    W1 = W0.copy()
    W1[:, 4] = 0.0  # column 5 (1-based) is already eliminated
    sks = [rhqr.Sketch(rhqr.SRHT, n, m, l, seed=s) for s in (1, 2)]
    b = rhqr.Batch([(sks[0], to_gpu(W0)), (sks[1], to_gpu(W1))])
    outs = b.factor()
    assert b.status() == [0, 5]
    ref = orq.rhqr_left(W1, osk.Sketch(osk.SRHT, n, m, l, seed=2))
    assert ref["info"] == 5
    assert rel(to_np(outs[1]["R"]), ref["R"]) < 1e-12
    b.close()


def test_batch_c4_shapes_fp32_bounds():
    """Problems of the batched workload's kind (n = 2^k, m in [16, 128], l = 4m,
    cond log-uniform in 1e2..1e12, float32), fewer and smaller so the oracle's
    metrics stay cheap: e_fact and e_orth within the float32 tolerance."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    rng = np.random.default_rng(0)
    shapes = []
    for i in range(12):
        k = int(rng.integers(14, 17))
        m = int(rng.integers(16, 129))
        shapes.append((1 << k, m, 4 * m, 1000 + i, float(rng.uniform(2, 12))))
    probs = []
    for n, m, l, seed, kap in shapes:
        W = synthetic_matrix(n, m, kap, seed=seed)
        probs.append((W, rhqr.Sketch(rhqr.SRHT, n, m, l, seed=seed)))
    d = [np.abs(W).max(axis=0) for W, _ in probs]
    b = rhqr.Batch([(sk, to_gpu(W / dd, torch.float32)) for (W, sk), dd in zip(probs, d)],
                   panel=16)
    outs = b.factor(graph=True)
    torch.cuda.synchronize()
    assert b.status() == [0] * len(probs)
    for (W, sk), dd, o, (n, m, l, seed, kap) in zip(probs, d, outs, shapes):
        Wt = (W / dd).astype(np.float32).astype(np.float64)  # the rounded input
        U, S, T, R = (to_np(o[k]) for k in ("U", "S", "T", "R"))
        Q = orq.thin_q(U, T, m)
        ef = metrics.fact_error(Wt, Q, R)
        eo = metrics.orth_error(osk.rh_sketch(Q, osk.Sketch(osk.SRHT, n, m, l, seed=seed)))
        log(f"  n={n} m={m} cond=1e{kap:.1f}: e_fact {ef:.2e} e_orth {eo:.2e}")
        assert ef <= 1e-5 and eo <= 1e-5
    b.close()


@pytest.mark.parametrize("panel", [0, 16])
@pytest.mark.parametrize("dt", ["float64", "float32", "float16"])
def test_batch_thin_q_bitwise_equals_single(dt, panel):
    """rhqr_batch_thin_q after the batch: every problem's thin Q (Sec. 3.2)
    equals the one rhqr_factor forms with want_q, bitwise (same kernels on the
    same U, S, T); one problem is skipped (NULL Q) and must stay untouched."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    from paper_2405_10923_amd.rhqr import colmajor_empty
    tdt = getattr(torch, dt)
    probs = _inputs(torch, tdt)
    log(f"batch thin Q {dt} panel={panel}: {len(probs)} problems")
    b = rhqr.Batch([(sk, to_gpu(W, tdt)) for W, sk, _ in probs], panel=panel)
    b.factor()
    Qs = [colmajor_empty(W.shape[0], W.shape[1], tdt, "cuda") for W, _, _ in probs]
    for Q in Qs:
        Q.fill_(7.0)
    skip = 3
    import ctypes as C
    k = len(Qs)
    ptrs = (C.c_void_p * k)(*[None if i == skip else Q.data_ptr() for i, Q in enumerate(Qs)])
    lds = (C.c_int64 * k)(*[Q.stride(1) for Q in Qs])
    assert rhqr.lib().rhqr_batch_thin_q(b.h, ptrs, lds, rhqr._stream()) == 0
    torch.cuda.synchronize()
    assert b.status() == [0] * k
    for i, ((W, sk, shp), Q) in enumerate(zip(probs, Qs)):
        if i == skip:
            assert bool((Q == 7.0).all()), shp
            continue
        ref = rhqr.factor(sk, to_gpu(W, tdt), panel=panel, want_q=True)
        torch.cuda.synchronize()
        assert torch.equal(Q, ref["Q"]), shp
    # the Python wrapper on its own buffers
    Qw = b.thin_q()
    torch.cuda.synchronize()
    for i, Q in enumerate(Qw):
        if i != skip:
            assert torch.equal(Q, Qs[i])
    b.close()


# Gaussian batches: Omega drawn by the test (the oracle's draw) and handed to
# both sides; one sketch kind per batch
GSHAPES = [(5000, 12, 48, 1), (3 * 4096 + 777, 24, 96, 3), (300, 7, 40, 4), (2 * 4096 + 5, 40, 130, 7)]


def _gauss_inputs(shapes=GSHAPES, kappa=3.0):
    from paper_2405_10923_amd import rhqr
    probs = []
    for n, m, l, seed in shapes:
        W = synthetic_matrix(n, m, kappa, seed=seed)
        osketch = osk.Sketch(osk.GAUSS, n, m, l, seed=seed + 200)
        sk = rhqr.Sketch(rhqr.GAUSS, n, m, l, seed=seed + 200, omega=to_gpu(osketch.omega))
        probs.append((W, sk, osketch, (n, m, l, seed)))
    return probs


@pytest.mark.parametrize("panel", [0, 16, (8, 32)])
@pytest.mark.parametrize("dt", ["float64", "float32", "bfloat16"])
def test_batch_gauss_bitwise_equals_single(dt, panel):
    """A batch of Gaussian-sketch problems: per problem the single-problem
    pre-sketch and tall workgroups, so every factor equals rhqr_factor's
    bitwise; the hipGraph form replays to the same bits."""
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    tdt = getattr(torch, dt)
    probs = _gauss_inputs()
    log(f"gaussian batch {dt} panel={panel}: {len(probs)} problems")
    pn, outer = _sched(panel)
    b = rhqr.Batch([(sk, to_gpu(W, tdt)) for W, sk, _, _ in probs], panel=pn, outer=outer)
    outs = b.factor()
    torch.cuda.synchronize()
    assert b.status() == [0] * len(probs)
    eager = [{k: o[k].clone() for k in ("U", "S", "T", "R")} for o in outs]
    for (W, sk, _, shp), o in zip(probs, outs):
        log(f"  single {shp}")
        ref = rhqr.factor(sk, to_gpu(W, tdt), panel=pn, outer=outer)
        torch.cuda.synchronize()
        for k in ("U", "S", "T", "R"):
            assert torch.equal(o[k], ref[k]), (shp, k)
    if dt == "float64":
        for rep in range(2):
            for (W, _, _, _), o in zip(probs, outs):
                o["U"].copy_(to_gpu(W, tdt))
            b.factor(graph=True)
            torch.cuda.synchronize()
            for e, o in zip(eager, outs):
                for k in e:
                    assert torch.equal(o[k], e[k]), (rep, k)
    b.close()


def test_batch_gauss_f64_matches_oracle():
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    probs = _gauss_inputs(kappa=2.0)
    b = rhqr.Batch([(sk, to_gpu(W)) for W, sk, _, _ in probs], panel=16)
    outs = b.factor()
    torch.cuda.synchronize()
    for (W, _, osketch, (n, m, l, _)), o in zip(probs, outs):
        log(f"  oracle gaussian {n} {m} {l}")
        ref = orq.rhqr_left(W, osketch)
        for k in ("U", "S", "T", "R"):
            assert rel(to_np(o[k]), ref[k]) < 1e-12, (n, m, l, k)
    b.close()


def test_batch_rejects_mixed_sketch_kinds():
    torch = cuda_or_skip()
    from paper_2405_10923_amd import rhqr
    (W0, sk0, _, _), = _gauss_inputs(shapes=[(5000, 12, 48, 1)])
    sk1 = rhqr.Sketch(rhqr.SRHT, 4096, 8, 32, seed=3)
    W1 = synthetic_matrix(4096, 8, 2.0, seed=3)
    with pytest.raises(rhqr.RHQRError):
        rhqr.Batch([(sk0, to_gpu(W0)), (sk1, to_gpu(W1))])
