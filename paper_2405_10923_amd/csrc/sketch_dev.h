// Device code of the multi-column SRHT sketch (RHSketch, Alg. 1), shared by
// the single-problem kernels (sketch.hip) and the batched kernels
// (batched.hip).
#pragma once
#include "common.h"

namespace {

// ------------------------------------------------------------ RHSketch, SRHT
// Grid (gt, k): workgroup (g, c) transforms tiles t = g, g+gt, ... of column c
// and accumulates its contribution to each of the l samples; part[c][g][q].
// Later tiles' loads are issued before the current tile's transform.  512
// threads transform one tile (TILE rows) per step, so two workgroups fit on a
// compute unit and overlap one's loads with the other's transform.
//
// The 12 index bits of a tile are split three ways.  A thread holds 8 values:
// its 16-byte vectors' elements and its vectors, i.e. the low VL bits
// (VL = log2 of the elements per vector) and the bits above the 9 bits of the
// thread index; their butterflies run in registers.  The thread-index bits
// [VL, VL + 9) go through LDS: two radix-16 passes over [VL, VL + 4) and
// [VL + 4, VL + 8), and the last bit, VL + 8, is folded into the sample
// reads (out[r] = s[r without the bit] +/- s[r with it]).  The butterflies
// over distinct bits commute, so this is the same transform as three radix-16
// passes over the whole tile, up to rounding, with 24 % less LDS traffic.
constexpr int SK_TPB = 512, SK_TPW = 1;

// one radix-16 pass over the tile bits [sh, sh + 4), 256 threads of 16 values
template <typename A> __device__ __forceinline__ void fwht_sk_pass(A *s, int sh) {
  lds_barrier();
  const int g = threadIdx.x;
  if (g < TILE / 16) {
    const int lo = g & ((1 << sh) - 1);
    const int hi = g >> sh;
    const int base = lo + (hi << (sh + 4));
    A v[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) v[k] = s[tpad(base + (k << sh))];
    fwht16(v);
#pragma unroll
    for (int k = 0; k < 16; ++k) s[tpad(base + (k << sh))] = v[k];
  }
}

// Row groups whose loads are in flight ahead of the one being transformed:
// about 128 bytes of the column per thread for every storage type.
template <typename ST> constexpr int sk_prefetch() { return sizeof(ST) == 8 ? 2 : sizeof(ST) == 4 ? 4 : 8; }

// Each workgroup walks the row groups g = gb, gb + gt, ... of column c (the
// i-th of its groups is gb + i gt).  Groups that lie entirely inside the n
// rows of a 16-byte aligned column are loaded PF at a time; LDS-only barriers
// keep the later groups' loads in flight across the butterflies of the
// earlier ones.  The ragged last group (and every group of an unaligned
// column) is loaded element by element.
template <typename ST, typename AT, int QA, int PF = sk_prefetch<ST>()>
__device__ __forceinline__ void srht_cols_block(const ST *__restrict__ X, int64_t ldx, int64_t n,
                                                int32_t m, int32_t l, int64_t ngroups, int gt,
                                                const uint64_t *__restrict__ signs,
                                                const int32_t *__restrict__ rows,
                                                double *__restrict__ part, int aligned, int gb,
                                                int c) {
  constexpr int VEC = 16 / sizeof(ST);
  constexpr int ROWS = TILE * SK_TPW;
  constexpr int NV = ROWS / (SK_TPB * VEC);
  constexpr int NE = NV * VEC;
  constexpr int VL = VEC == 2 ? 1 : VEC == 4 ? 2 : 3;
  constexpr int FB = VL + 8;  // the folded bit
  static_assert(SK_TPW == 1 && SK_TPB == 512 && TILE == 4096 && NE == 8,
                "3 register bits, 9 thread-index bits");
  static_assert(VEC <= 32, "a thread's rows must share one 32-bit sign word");
  __shared__ AT s[TILE_PAD];
  const ST *x = X + (int64_t)c * ldx;
  // sign bit i is bit i % 32 of 32-bit word i / 32 (the 64-bit words, little-endian)
  const uint32_t *__restrict__ sg32 = reinterpret_cast<const uint32_t *>(signs);
  // per sample: the padded positions of its tile row without and with the
  // folded bit, whether that bit is set, and its tile-index bits
  double acc[QA];
  int r0q[QA], r1x[QA];
  bool fneg[QA];
  uint64_t r1q[QA];
#pragma unroll
  for (int a = 0; a < QA; ++a) {
    acc[a] = 0.0;
    const int q = threadIdx.x + SK_TPB * a;
    const int32_t r = q < l ? rows[q] : 0;
    const int r2 = r & (TILE - 1);
    r0q[a] = tpad(r2 & ~(1 << FB));
    r1x[a] = tpad(r2 | (1 << FB));
    fneg[a] = (r2 >> FB) & 1;
    r1q[a] = (uint64_t)(r >> TILE_LOG);
  }
  const int64_t cnt = gb < ngroups ? (ngroups - 1 - gb) / gt + 1 : 0;
  const int64_t nfullg = n / ROWS;  // groups entirely inside the n rows
  const int64_t cntf = !aligned ? 0 : (gb < nfullg ? (nfullg - 1 - gb) / gt + 1 : 0);
  // signed, transformed group g, then its samples into acc
  // xs: the group's values, raw (16-byte words as loaded, decoded here) or
  // already in AT
  auto transform = [&](int64_t g, const auto &xs, const uint32_t (&ws)[NV]) {
    const int64_t base = g * ROWS;
    AT t[NE];  // t[VEC v + e]: row VEC (tid + SK_TPB v) + e of the group
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t i0 = base + VEC * (threadIdx.x + SK_TPB * v);
      AT xd[VEC];
      if constexpr (std::is_same<std::decay_t<decltype(xs[0])>, u32x4>::value) {
        vdecode<ST, AT>(xs[v], xd);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xd[e] = xs[v][e];
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t r = i0 + e;
        AT val = (r >= m && r < n) ? xd[e] : (AT)0;
        if ((ws[v] >> (r & 31)) & 1u) val = -val;
        t[v * VEC + e] = val;
      }
    }
    // the bits of the index VEC v + e are tile bits: their butterflies here
#pragma unroll
    for (int h = 1; h < NE; h <<= 1)
#pragma unroll
      for (int i = 0; i < NE; ++i)
        if ((i & h) == 0) {
          const AT a = t[i], b = t[i + h];
          t[i] = a + b;
          t[i + h] = a - b;
        }
    lds_barrier();  // the previous group's samples have been read
#pragma unroll
    for (int v = 0; v < NV; ++v)
#pragma unroll
      for (int e = 0; e < VEC; ++e) s[tpad(VEC * (threadIdx.x + SK_TPB * v) + e)] = t[v * VEC + e];
    fwht_sk_pass(s, VL);
    fwht_sk_pass(s, VL + 4);
    lds_barrier();
#pragma unroll
    for (int a = 0; a < QA; ++a) {
      const int q = threadIdx.x + SK_TPB * a;
      if (q < l) {
        const double h0 = (double)s[r0q[a]], h1 = (double)s[r1x[a]];
        const double hv = fneg[a] ? h0 - h1 : h0 + h1;
        acc[a] += (__popcll(r1q[a] & (uint64_t)g) & 1) ? -hv : hv;
      }
    }
  };
  // PF groups per iteration, all their loads issued first (as raw 16-byte
  // words), then transformed in order: each transform waits only for its own
  // group while the later groups' loads are still in flight.  No load is
  // carried across iterations (the compiler drains every outstanding load at
  // a loop header that has loads in flight from the back edge).
  const int64_t cntp = cntf / PF * PF;
  for (int64_t i0 = 0; i0 < cntp; i0 += PF) {
    u32x4 xv[PF][NV];
    uint32_t wd[PF][NV];
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) {
      const int64_t base = (gb + (i0 + sl) * (int64_t)gt) * ROWS;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t r0 = base + VEC * (threadIdx.x + SK_TPB * v);
        xv[sl][v] = vraw_nt(x + r0);
        wd[sl][v] = sg32[r0 >> 5];
      }
    }
#pragma unroll
    for (int sl = 0; sl < PF; ++sl) transform(gb + (i0 + sl) * (int64_t)gt, xv[sl], wd[sl]);
  }
  // the remaining groups one at a time: full ones with vector loads, the
  // ragged last one (or any group of an unaligned column) element by element
  for (int64_t i = cntp; i < cnt; ++i) {
    const int64_t g = gb + i * (int64_t)gt;
    const int64_t base = g * ROWS;
    AT xs[NV][VEC];
    uint32_t ws[NV];
    const bool vec = i < cntf;  // uniform
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t i0 = base + VEC * (threadIdx.x + SK_TPB * v);
      if (vec) {
        vload<ST, AT, true>(x + i0, xs[v]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xs[v][e] = (i0 + e < n) ? cvt_in<AT>(x[i0 + e]) : (AT)0;
      }
      ws[v] = i0 < n ? sg32[i0 >> 5] : 0u;
    }
    transform(g, xs, ws);
  }
#pragma unroll
  for (int a = 0; a < QA; ++a) {
    const int q = threadIdx.x + SK_TPB * a;
    if (q < l) part[((int64_t)c * gt + gb) * l + q] = acc[a];
  }
}

// Y[:, c] = [X_{1:m,c}; scale * sum_g part[c][g][:]]
template <typename ST>
__device__ __forceinline__ void sketch_finish_one(const ST *__restrict__ X, int64_t ldx, int32_t m,
                                                  int32_t l, int gt, const double *__restrict__ part,
                                                  double scale, double *__restrict__ Y, int64_t ldy,
                                                  int k, int c) {
  if (k >= m + l) return;
  double v;
  if (k < m) {
    v = cvt_in<double>(X[(int64_t)c * ldx + k]);
  } else {
    const int q = k - m;
    const double *p = part + (int64_t)c * gt * l + q;
    double s = 0.0;
    for (int g = 0; g < gt; ++g) s += p[(int64_t)g * l];
    v = s * scale;
  }
  Y[(int64_t)c * ldy + k] = v;
}

}  // namespace
