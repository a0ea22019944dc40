"""Philox4x64-10 (Salmon, Moraes, Dror & Shaw, "Parallel random numbers: as easy
as 1, 2, 3", SC'11), vectorised over numpy uint64 arrays.

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

The paper draws its embeddings "from a seeded random number generator" without
naming one (Sec. 2.3, Gaussian OSE paragraph; SRHT paragraph).  This project
fixes Philox4x64-10 with key = (seed, stream) and counter = (block, 0, 0, 0).
The implementation below is written from the published round function:

    (hi0, lo0) = mulhilo(M0, x0);  (hi1, lo1) = mulhilo(M1, x2)
    x <- (hi1 ^ x1 ^ k0,  lo1,  hi0 ^ x3 ^ k1,  lo0)
    k <- k + (W0, W1)          (between rounds)

It is pinned against numpy's independent ``numpy.random.Philox`` bit generator
in ``tests/test_oracle_rng.py``.
"""
import numpy as np

M0 = np.uint64(0xD2E7470EE14C6C93)
M1 = np.uint64(0xCA5A826395121157)
W0 = np.uint64(0x9E3779B97F4A7C15)
W1 = np.uint64(0xBB67AE8584CAA73B)
_LO32 = np.uint64(0xFFFFFFFF)
_S32 = np.uint64(32)

# stream identifiers (second key word) used by the sketch draws
STREAM_SIGNS = 0
STREAM_ROWKEYS = 1
STREAM_GAUSS = 2


def mulhilo(a, b):
    """Full 64x64 -> 128-bit product of uint64 arrays, returned as (hi, lo)."""
    a = np.asarray(a, dtype=np.uint64)
    b = np.asarray(b, dtype=np.uint64)
    a_lo, a_hi = a & _LO32, a >> _S32
    b_lo, b_hi = b & _LO32, b >> _S32
    ll = a_lo * b_lo
    hl = a_hi * b_lo
    lh = a_lo * b_hi
    hh = a_hi * b_hi
    # each partial product is < 2**64; the middle sum cannot overflow
    mid = (ll >> _S32) + (hl & _LO32) + lh
    hi = hh + (hl >> _S32) + (mid >> _S32)
    lo = a * b  # wraps modulo 2**64
    return hi, lo


def philox4x64_10(ctr, key):
    """Ten Philox rounds.  ``ctr`` is a 4-tuple and ``key`` a 2-tuple of uint64
    arrays (broadcastable).  Returns the four output words as uint64 arrays."""
    with np.errstate(over="ignore"):
        x0, x1, x2, x3 = (np.asarray(c, dtype=np.uint64) for c in ctr)
        k0, k1 = (np.asarray(k, dtype=np.uint64) for k in key)
        for r in range(10):
            if r > 0:
                k0 = k0 + W0
                k1 = k1 + W1
            hi0, lo0 = mulhilo(M0, x0)
            hi1, lo1 = mulhilo(M1, x2)
            x0, x1, x2, x3 = hi1 ^ x1 ^ k0, lo1, hi0 ^ x3 ^ k1, lo0
    return x0, x1, x2, x3


def words(seed, stream, count):
    """The first ``count`` 64-bit words of stream ``stream``: word i is output
    word (i mod 4) of block i // 4, block b using counter (b, 0, 0, 0)."""
    nblk = (count + 3) // 4
    b = np.arange(nblk, dtype=np.uint64)
    z = np.zeros_like(b)
    out = philox4x64_10((b, z, z, z), (np.uint64(seed), np.uint64(stream)))
    return np.stack(out, axis=1).reshape(-1)[:count]
