#!/usr/bin/env python3
"""Benchmark: left-looking RHQR (Alg. 4) of a 2^22 x 256 matrix on one MI355X.

Workload: W = G diag(s) V, G iid N(0,1), singular values logspaced 1..1e-14,
V Haar-orthogonal; SRHT sketch with l = 1024, seed 0.  One step is one
rhqr_factor call: pre-sketch Psi W, the 256-column loop (refresh + re-sketch
pass, float64 sketch-space step), outputs U (in place of W), S, T, R.  The
input is restored from a pristine copy between steps, outside the timed
events.  Mixed precision (n-row data in float32 / float16 / bfloat16 with
float32 accumulation; unit-max column scaling before rounding) is timed on
the same workload and gated on ||W~ - QR||/||W~|| <= 1e-2 and
||(Psi Q)^t Psi Q - I||_2 <= 1e-2.

value = B_alg / t for float64, B_alg = 8 (n-m) [m(m-1)/2 + 3m] bytes (the
paper's algorithm: U_{j-1} read by the refresh of column j, plus the
pre-sketch read, the column read and the u_j write).

Prints ONE JSON line.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "RHQR GB/s (% HBM roofline), mixed vs FP64 at ||W-QR||/||W|| <= 1e-2"
HBM_PEAK_GBS = 8000.0


def b_alg(n, m, b):
    return b * (n - m) * (m * (m - 1) / 2 + 3 * m)


def tall_bytes_per_launch_avg(n, m, l, b):
    """Algorithmic bytes of the refresh + re-sketch kernel, averaged over its
    m-1 launches: launch j reads the j-1 stored columns of U, the raw column
    j-1 and w_j, writes u_{j-1} and the raw refreshed column j (j+3 columns of
    n-m rows), reads the sign bits and writes one l-vector of partials per
    4096-row tile."""
    ntiles = (n + 4095) // 4096
    N = 1 << (n - 1).bit_length()
    tot = 0.0
    for j in range(1, m):
        tot += (j + 3) * b * (n - m) + ntiles * l * 8 + N / 8
    return tot / (m - 1)


def cpu_baseline(n, l, kappa, ncols=8, seed=0):
    """The CPU oracle, untuned, on a bounded sample: the first ``ncols``
    columns of the workload's matrix shape (n rows), head m = ncols."""
    import numpy as np
    from oracle import sketch as osk, rhqr as orq
    from paper_2405_10923_amd.inputs import synthetic_matrix
    try:
        from threadpoolctl import threadpool_info
        threads = max([i.get("num_threads", 1) for i in threadpool_info()] + [1])
    except Exception:
        threads = os.cpu_count() or 1
    W = synthetic_matrix(n, ncols, kappa, seed=seed)
    t0 = time.perf_counter()
    sk = osk.Sketch(osk.SRHT, n, ncols, l, seed=seed)
    orq.rhqr_left(W, sk)
    dt = time.perf_counter() - t0
    gbs = b_alg(n, ncols, 8) / dt / 1e9
    return {"value": gbs, "unit": "GB/s", "cores": int(threads), "kind": "oracle",
            "sample": f"float64 left-looking RHQR of a {n} x {ncols} slice of the workload "
                      f"(SRHT l={l}, head {ncols}), sketch draw included; {dt:.1f} s"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--n", type=int, default=1 << 22)
    ap.add_argument("--m", type=int, default=256)
    ap.add_argument("--l", type=int, default=1024)
    ap.add_argument("--kappa", type=float, default=14.0)
    ap.add_argument("--dtypes", default="float64,float32,float16,bfloat16")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-cols", type=int, default=8)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "row-sharded design is described but not built.", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch
    from paper_2405_10923_amd import rhqr
    from paper_2405_10923_amd.inputs import synthetic_matrix_torch

    n, m, l, kappa = args.n, args.m, args.l, args.kappa
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    print(f"# workload n={n} m={m} l={l} cond=1e{kappa:g}", file=sys.stderr, flush=True)
    W64 = synthetic_matrix_torch(n, m, kappa, seed=0, device="cuda")
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=0)
    res = {}
    roof = None
    for name in args.dtypes.split(","):
        dt = getattr(torch, name)
        b = torch.finfo(dt).bits // 8
        if dt == torch.float64:
            Wsrc = W64
            d = None
        else:
            d = W64.abs().amax(dim=0)
            Wsrc = torch.empty((m, n), dtype=dt, device=dev).t()
            Wsrc.copy_(W64 / d)
        Ww = torch.empty((m, n), dtype=dt, device=dev).t()
        bufs = rhqr.FactorBuffers(sk, dt, m, want_q=False)
        for _ in range(args.warmup):
            Ww.copy_(Wsrc)
            rhqr.factor(sk, Ww, bufs=bufs)
        torch.cuda.synchronize()
        prof = dt == torch.float64
        if prof:
            rhqr.profile_begin()
        evs = []
        for _ in range(args.steps):
            Ww.copy_(Wsrc)
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e0.record()
            rhqr.factor(sk, Ww, bufs=bufs)
            e1.record()
            evs.append((e0, e1))
        torch.cuda.synchronize()
        ms = [a.elapsed_time(c) for a, c in evs]
        step_ms = float(np.mean(ms))
        if prof:
            tall_ms, launches = rhqr.profile_end()
            avg_ms = tall_ms / max(launches, 1)
            avg_bytes = tall_bytes_per_launch_avg(n, m, l, b)
            ach = avg_bytes / (avg_ms * 1e-3) / 1e9
            roof = {"bound": "hbm", "achieved": round(ach, 1), "peak": HBM_PEAK_GBS,
                    "unit": "GB/s", "frac": round(ach / HBM_PEAK_GBS, 4), "traffic": None,
                    "kernel": "k_tall<double,SRHT> (refresh + re-sketch pass)",
                    "avg_launch_ms": round(avg_ms, 4), "launches": launches,
                    "alg_bytes_per_launch": avg_bytes}
        # accuracy of one more factorization with Q (untimed)
        Ww.copy_(Wsrc)
        bq = rhqr.FactorBuffers(sk, dt, m, want_q=True)
        out = rhqr.factor(sk, Ww, want_q=True, bufs=bq)
        Q, R = out["Q"], out["R"]
        Wt = Wsrc.to(torch.float64)
        ef = float(torch.linalg.norm(Wt - Q.to(torch.float64) @ R) / torch.linalg.norm(Wt))
        Y = rhqr.sketch(sk, Q)
        G = (Y.t() @ Y).cpu().numpy()
        eo = float(np.linalg.norm(G - np.eye(m), 2))
        info = rhqr.status(out["ws"])
        del bq, out, Q, Y, Wt
        gbs = b_alg(n, m, b) / (step_ms * 1e-3) / 1e9
        res[name] = {"ms_per_step": round(step_ms, 3), "GBps_alg": round(gbs, 1),
                     "hbm_frac_alg": round(gbs / HBM_PEAK_GBS, 4), "e_fact": ef, "e_orth": eo,
                     "info": info, "factorizations_per_s": round(1000.0 / step_ms, 3)}
        print(f"# {name}: {step_ms:.2f} ms/step  {gbs:.0f} GB/s(alg)  e_fact {ef:.2e} "
              f"e_orth {eo:.2e}", file=sys.stderr, flush=True)
        del Ww, Wsrc, bufs
        torch.cuda.empty_cache()

    f64 = res.get("float64")
    mixed = {}
    for k, v in res.items():
        if k == "float64":
            continue
        v = dict(v)
        if f64:
            v["speedup_vs_f64"] = round(f64["ms_per_step"] / v["ms_per_step"], 3)
        v["meets_1e-2"] = bool(v["e_fact"] <= 1e-2 and v["e_orth"] <= 1e-2)
        mixed[k] = v
    head = f64 if f64 else next(iter(res.values()))
    line = {
        "metric": METRIC,
        "value": head["GBps_alg"],
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if f64 else args.dtypes.split(",")[0],
        "data": "synthetic",
        "config": {"workload": f"RHQR left-looking, W {n}x{m} cond 1e{kappa:g} "
                               f"(G diag(s) V), SRHT l={l}, seed 0",
                   "n": n, "m": m, "l": l, "sketch": "srht",
                   "e_fact": head["e_fact"], "e_orth": head["e_orth"],
                   "hbm_frac_alg": head["hbm_frac_alg"]},
        "roofline": roof,
        "mixed": mixed,
    }
    if not args.no_cpu:
        line["cpu_baseline"] = cpu_baseline(n, l, kappa, ncols=args.cpu_cols)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
