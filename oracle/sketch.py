"""Sketching matrices of Sec. 2.3 and the sketching routine RHSketch (Alg. 1).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__.py``).

Psi (eq. psi, Sec. 3.1) keeps the first m rows of a vector and applies an
l x (n-m) embedding Omega to the remaining n-m rows:

    Psi = [ I_m  0 ; 0  Omega ]  in R^{(l+m) x n}.

Readings fixed by this project (the paper leaves them open):

* SRHT length.  The Walsh-Hadamard transform needs a power-of-two length, so
  Omega acts on R^N, N = 2^ceil(log2 n): tail row i (m <= i < n) is coordinate
  i of R^N, the head coordinates and the padding n..N-1 are zero.  With the
  scale sqrt(N/l) of the SRHT paragraph of Sec. 2.3 this is an SRHT of R^N
  restricted to the tail coordinates.
* Hadamard order: natural (Sylvester) order, H_1 = [[1,1],[1,-1]],
  H_{p+1} = [[H_p, H_p],[H_p, -H_p]] (appendix, proof of Lemma srht).
* Order of operations: scale, flip signs, Hadamard transform, normalise by
  N^{-1/2}, sample -- the order Lemma srht analyses.
* Randomness (Philox4x64-10, key = (seed, stream)):
    - sign of coordinate i: bit (i mod 64) of word floor(i/64) of stream 0,
      a set bit meaning -1;
    - row sample: key_i = word i of stream 1 for i < N; the l rows are the
      indices of the l smallest pairs (key_i, i), i.e. a uniform draw without
      replacement, listed in increasing order;
    - Gaussian entry (k, i) of Omega (column-major index e = k + l*i): words
      2e, 2e+1 of stream 2 -> u1 = ((a >> 11) + 1) 2^-53 in (0, 1],
      u2 = (b >> 11) 2^-53 in [0, 1); g = sqrt(-2 ln u1) cos(2 pi u2)
      (Box-Muller); Omega_{k,i} = g / sqrt(l), entries N(0, 1/l) as in the
      Gaussian OSE paragraph of Sec. 2.3.
"""
import math

import numpy as np

from . import philox

SRHT = "srht"
GAUSS = "gauss"
IDENTITY = "identity"


def next_pow2(n):
    return 1 << max(0, (int(n) - 1).bit_length())


def srht_signs(seed, N):
    """Random signs D (Sec. 2.3, SRHT paragraph) for coordinates 0..N-1."""
    nw = (N + 63) // 64
    w = philox.words(seed, philox.STREAM_SIGNS, nw)
    i = np.arange(N, dtype=np.uint64)
    bits = (w[i >> np.uint64(6)] >> (i & np.uint64(63))) & np.uint64(1)
    return np.where(bits == 1, -1.0, 1.0)


def srht_rows(seed, N, l):
    """l of the N rows of the identity drawn uniformly without replacement
    (the sampling matrix P of the SRHT paragraph), in increasing order."""
    if not 0 < l <= N:
        raise ValueError("need 0 < l <= N")
    keys = philox.words(seed, philox.STREAM_ROWKEYS, N)
    order = np.lexsort((np.arange(N), keys))  # by key, ties by index
    return np.sort(order[:l]).astype(np.int64)


def gaussian_omega(seed, l, ntail):
    """Gaussian embedding Omega = G / sqrt(l), G iid N(0,1) (Sec. 2.3)."""
    cnt = l * ntail
    w = philox.words(seed, philox.STREAM_GAUSS, 2 * cnt).reshape(cnt, 2)
    a, b = w[:, 0], w[:, 1]
    u1 = ((a >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * 2.0 ** -53
    u2 = (b >> np.uint64(11)).astype(np.float64) * 2.0 ** -53
    g = np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)
    # column-major: entry (k, i) is element k + l*i
    return (g / math.sqrt(l)).reshape(ntail, l).T.copy()


def fwht(x):
    """Unnormalised Walsh-Hadamard transform H_p x along axis 0, natural order,
    by the butterfly recursion H_{p+1} = [[H_p, H_p], [H_p, -H_p]]."""
    x = np.array(x, dtype=np.float64, copy=True)
    N = x.shape[0]
    if N & (N - 1):
        raise ValueError("length must be a power of two")
    rest = x.shape[1:]
    h = 1
    while h < N:
        v = x.reshape((N // (2 * h), 2, h) + rest)
        a = v[:, 0].copy()
        b = v[:, 1]
        v[:, 0] = a + b
        v[:, 1] = a - b
        h *= 2
    return x


class Sketch:
    """The draw of Psi for an n x m problem: kind, sizes and the random data."""

    def __init__(self, kind, n, m, l, seed=0, omega=None):
        self.kind, self.n, self.m, self.l, self.seed = kind, int(n), int(m), int(l), seed
        if not (0 < self.m < self.n):
            raise ValueError("need 0 < m < n")
        self.N = next_pow2(self.n)
        self.signs = self.rows = self.omega = None
        if kind == SRHT:
            self.signs = srht_signs(seed, self.N)
            self.rows = srht_rows(seed, self.N, self.l)
        elif kind == GAUSS:
            self.omega = (gaussian_omega(seed, self.l, self.n - self.m)
                          if omega is None else np.asarray(omega, dtype=np.float64))
        elif kind == IDENTITY:
            self.l = self.n - self.m
        else:
            raise ValueError(kind)

    @property
    def rows_out(self):
        return self.l + self.m

    def omega_apply(self, X2):
        """Omega @ X2 for the n-m tail rows X2 (SRHT in the order of Lemma srht)."""
        X2 = np.asarray(X2, dtype=np.float64)
        if self.kind == IDENTITY:
            return X2.copy()
        if self.kind == GAUSS:
            return self.omega @ X2
        N, m, n, l = self.N, self.m, self.n, self.l
        v = np.zeros((N,) + X2.shape[1:])
        v[m:n] = X2
        v = math.sqrt(N / l) * v                                 # scale
        v = self.signs.reshape((N,) + (1,) * (v.ndim - 1)) * v    # flip signs
        v = fwht(v)                                              # Hadamard
        v = v / math.sqrt(N)                                     # normalise
        return v[self.rows]                                      # sample


def rh_sketch(X, sk):
    """RHSketch (Alg. 1): [X_{1:m}; Omega X_{m+1:n}] for X with n rows."""
    X = np.asarray(X, dtype=np.float64)
    return np.concatenate([X[: sk.m], sk.omega_apply(X[sk.m:])], axis=0)
