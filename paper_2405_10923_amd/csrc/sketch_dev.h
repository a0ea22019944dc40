// Device code of the multi-column SRHT sketch (RHSketch, Alg. 1), shared by
// the single-problem kernels (sketch.hip) and the batched kernels
// (batched.hip).
#pragma once
#include "common.h"

namespace {

// ------------------------------------------------------------ RHSketch, SRHT
// Grid (gt, k): workgroup (g, c) transforms tiles t = g, g+gt, ... of column c
// and accumulates its contribution to each of the l samples; part[c][g][q].
// The next tile's loads are issued before the current tile's transform.
// 1024 threads transform two consecutive tiles (2 TILE rows) per step; two
// workgroups per compute unit overlap one's loads with the other's transform.
constexpr int SK_TPB = 1024, SK_TPW = 2;

template <typename A> __device__ void fwht_two_tiles(A *s) {
#pragma unroll 1
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

// Each workgroup walks the row groups g = blockIdx.x, blockIdx.x + gt, ... of
// column blockIdx.y; the loads of group g + gt are issued before the transform
// of group g (LDS-only barriers keep them in flight), so HBM reads overlap the
// in-LDS butterflies.
template <typename ST, typename AT, int QA>
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
  __shared__ AT s[SK_TPW * TILE_PAD];
  const ST *x = X + (int64_t)c * ldx;
  double acc[QA];
#pragma unroll
  for (int a = 0; a < QA; ++a) acc[a] = 0.0;
  AT xv[NV][VEC];
  uint64_t wd[NV];
  auto fetch = [&](int64_t g) {
    const int64_t base = g * ROWS;
    const bool fast = aligned && base + ROWS <= n;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t i0 = base + VEC * (threadIdx.x + SK_TPB * v);
      if (fast) {
        vload<ST, AT, true>(x + i0, xv[v]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) xv[v][e] = (i0 + e < n) ? cvt_in<AT>(x[i0 + e]) : (AT)0;
      }
      wd[v] = i0 < n ? signs[i0 >> 6] : 0ull;
    }
  };
  int64_t g = gb;
  if (g < ngroups) fetch(g);
  for (; g < ngroups; g += gt) {
    const int64_t base = g * ROWS;
    lds_barrier();  // the previous group's samples have been read
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int li0 = VEC * (threadIdx.x + SK_TPB * v);
      const int64_t i0 = base + li0;
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t i = i0 + e;
        AT val = (i >= m && i < n) ? xv[v][e] : (AT)0;
        if ((wd[v] >> (i & 63)) & 1ull) val = -val;
        const int li = li0 + e;
        s[(li >> TILE_LOG) * TILE_PAD + tpad(li & (TILE - 1))] = val;
      }
    }
    if (g + gt < ngroups) fetch(g + gt);
    fwht_two_tiles(s);
    const uint64_t t0 = (uint64_t)g * SK_TPW;
#pragma unroll
    for (int a = 0; a < QA; ++a) {
      const int q = threadIdx.x + SK_TPB * a;
      if (q < l) {
        const int32_t r = rows[q];
        const int r2 = tpad(r & (TILE - 1));
        const uint64_t r1 = (uint64_t)(r >> TILE_LOG);
#pragma unroll
        for (int tt = 0; tt < SK_TPW; ++tt) {
          const double h = (double)s[tt * TILE_PAD + r2];
          acc[a] += (__popcll(r1 & (t0 + tt)) & 1) ? -h : h;
        }
      }
    }
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
