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
// compute unit (about 110 registers per lane, 35 KB of LDS in float64) and
// overlap one's loads with the other's transform.
constexpr int SK_TPB = 512, SK_TPW = 1;

template <typename A> __device__ __forceinline__ void fwht_sk_group(A *s) {
  // fully unrolled: no inner loop, so the waits for loads in flight across
  // the transform stay exact
#pragma unroll
  for (int pass = 0; pass < 3; ++pass) {
    lds_barrier();
    const int sh = 4 * pass;
    const int gg = threadIdx.x;
    if (gg < (TILE / 16) * SK_TPW) {
      A *st = s + (gg >> 8) * TILE_PAD;
      const int g = gg & 255;
      const int lo = g & ((1 << sh) - 1);
      const int hi = g >> sh;
      const int base = lo + (hi << (sh + 4));
      A v[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) v[k] = st[tpad(base + (k << sh))];
      fwht16(v);
#pragma unroll
      for (int k = 0; k < 16; ++k) st[tpad(base + (k << sh))] = v[k];
    }
  }
  lds_barrier();
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
  static_assert(NV >= 1, "tile too small for the vector width");
  static_assert(VEC <= 32, "a thread's rows must share one 32-bit sign word");
  __shared__ AT s[SK_TPW * TILE_PAD];
  const ST *x = X + (int64_t)c * ldx;
  // sign bit i is bit i % 32 of 32-bit word i / 32 (the 64-bit words, little-endian)
  const uint32_t *__restrict__ sg32 = reinterpret_cast<const uint32_t *>(signs);
  double acc[QA];
  int r2q[QA];
  uint64_t r1q[QA];
#pragma unroll
  for (int a = 0; a < QA; ++a) {
    acc[a] = 0.0;
    const int q = threadIdx.x + SK_TPB * a;
    const int32_t r = q < l ? rows[q] : 0;
    r2q[a] = tpad(r & (TILE - 1));
    r1q[a] = (uint64_t)(r >> TILE_LOG);
  }
  const int64_t cnt = gb < ngroups ? (ngroups - 1 - gb) / gt + 1 : 0;
  const int64_t nfullg = n / ROWS;  // groups entirely inside the n rows
  const int64_t cntf = !aligned ? 0 : (gb < nfullg ? (nfullg - 1 - gb) / gt + 1 : 0);
  // signed, transformed group g in LDS, then its samples into acc
  // xs: the group's values, raw (16-byte words as loaded, decoded here) or
  // already in AT
  auto transform = [&](int64_t g, const auto &xs, const uint32_t (&ws)[NV]) {
    const int64_t base = g * ROWS;
    lds_barrier();  // the previous group's samples have been read
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int li0 = VEC * (threadIdx.x + SK_TPB * v);
      const int64_t i0 = base + li0;
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
        const int li = li0 + e;
        s[(li >> TILE_LOG) * TILE_PAD + tpad(li & (TILE - 1))] = val;
      }
    }
    fwht_sk_group(s);
    const uint64_t t0 = (uint64_t)g * SK_TPW;
#pragma unroll
    for (int a = 0; a < QA; ++a) {
      const int q = threadIdx.x + SK_TPB * a;
      if (q < l) {
#pragma unroll
        for (int tt = 0; tt < SK_TPW; ++tt) {
          const double hv = (double)s[tt * TILE_PAD + r2q[a]];
          acc[a] += (__popcll(r1q[a] & (t0 + tt)) & 1) ? -hv : hv;
        }
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
