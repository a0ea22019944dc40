"""Autotuner of the blocked schedule: for a storage type and a problem size it
times rhqr_factor over a set of candidate schedules -- inner panel width,
outer panel width, transform tiles per workgroup of the refresh pass -- on a
synthetic matrix of that size on the current GPU, and records the fastest in
a JSON cache next to this file (tuned_schedules.json), which
``schedules.lookup`` reads.

    python -m paper_2405_10923_amd.autotune --shape 4194304x256:1024 --dtypes float64,float16

Problem sizes are bucketed by ceil(log2 n) and by m in powers of two, so one
entry serves the neighbouring sizes.  Every candidate computes the same
factorization (the schedules differ only in the order of the panel updates
and of the sketch partials' sums), so the choice is purely one of speed.
"""
import argparse
import json
import math
import os
import sys
import time

HERE = os.path.dirname(os.path.abspath(__file__))
CACHE = os.path.join(HERE, "tuned_schedules.json")

# (panel, outer, tpw); tpw 0 lets the library choose from n
CANDIDATES = [(8, 32, 0), (8, 32, 2), (8, 32, 4), (8, 16, 0), (4, 16, 0), (4, 32, 0),
              (16, 32, 0), (16, 0, 0), (16, 0, 2), (16, 0, 4), (8, 0, 0), (32, 0, 0)]


def bucket(n, m):
    """Cache key part for a problem size: ceil(log2 n) and the power of two
    at or above m."""
    return f"n2^{max(0, (int(n) - 1).bit_length())}|m{1 << max(0, (int(m) - 1).bit_length())}"


def key(dtype_name, n, m):
    return f"{dtype_name}|{bucket(n, m)}"


def load(path=None):
    path = path or CACHE
    try:
        with open(path) as fh:
            return json.load(fh)
    except (OSError, ValueError):
        return {}


def valid(cand, m, es):
    panel, outer, tpw = cand
    if panel > m:
        return False
    if es == 2 and tpw == 1:
        return False
    return outer == 0 or (outer > panel and outer % panel == 0 and outer <= 32)


def time_schedule(rhqr, torch, sk, Wsrc, cand, steps, warmup):
    """Mean ms of one factorization with schedule ``cand`` (HIP events), the
    input restored from ``Wsrc`` outside the timed events."""
    panel, outer, tpw = cand
    m = Wsrc.shape[1]
    W = rhqr.colmajor_empty(Wsrc.shape[0], m, Wsrc.dtype, Wsrc.device)
    bufs = rhqr.FactorBuffers(sk, Wsrc.dtype, m)
    evs = []
    for i in range(warmup + steps):
        W.copy_(Wsrc)
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record()
        rhqr.factor(sk, W, bufs=bufs, panel=panel, outer=outer, tpw=tpw)
        e1.record()
        if i >= warmup:
            evs.append((e0, e1))
    torch.cuda.synchronize()
    return sum(a.elapsed_time(b) for a, b in evs) / len(evs)


def tune(n, m, l, dtype_name, steps=3, warmup=1, candidates=None, log=print):
    """Time every valid candidate for an n x m factorization with an SRHT of
    l rows; returns (best entry, all timings)."""
    import torch
    from . import rhqr
    from .inputs import synthetic_matrix_torch
    dt = getattr(torch, dtype_name)
    es = torch.finfo(dt).bits // 8
    W64 = synthetic_matrix_torch(n, m, 8, seed=0, device="cuda")
    Wsrc = W64 if dt == torch.float64 else rhqr.colscale(W64, dt)[0]
    sk = rhqr.Sketch(rhqr.SRHT, n, m, l, seed=0)
    table = []
    for cand in candidates or CANDIDATES:
        if not valid(cand, m, es):
            continue
        ms = time_schedule(rhqr, torch, sk, Wsrc, cand, steps, warmup)
        table.append({"panel": cand[0], "outer": cand[1], "tpw": cand[2], "ms": round(ms, 4)})
        log(f"  {dtype_name} {n} x {m} l={l} panel={cand[0]} outer={cand[1]} tpw={cand[2]}: "
            f"{ms:.3f} ms")
    best = min(table, key=lambda e: e["ms"])
    del W64, Wsrc, sk
    torch.cuda.empty_cache()
    return dict(best, n=n, m=m, l=l, measured=time.strftime("%Y-%m-%d")), table


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--shape", action="append", required=True,
                    help="NxM:L (repeatable), e.g. 4194304x256:1024")
    ap.add_argument("--dtypes", default="float64,float32,float16,bfloat16")
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--cache", default=None)
    args = ap.parse_args()
    cache = load(args.cache)
    for shp in args.shape:
        nm, l = shp.split(":")
        n, m = (int(v) for v in nm.split("x"))
        for name in args.dtypes.split(","):
            best, table = tune(n, m, int(l), name, steps=args.steps,
                               log=lambda s: print(s, file=sys.stderr, flush=True))
            best["candidates"] = table
            cache[key(name, n, m)] = best
            print(f"# {key(name, n, m)} -> panel {best['panel']} outer {best['outer']} "
                  f"tpw {best['tpw']} ({best['ms']:.3f} ms)", file=sys.stderr, flush=True)
            with open(args.cache or CACHE, "w") as fh:
                json.dump(cache, fh, indent=1, sort_keys=True)
    print(json.dumps({k: {kk: v[kk] for kk in ("panel", "outer", "tpw", "ms")}
                      for k, v in cache.items()}))


if __name__ == "__main__":
    main()
