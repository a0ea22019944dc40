// Device code of one column of the left-looking RHQR loop (Alg. 4 with
// RHVector, Alg. 2), shared by the single-problem kernels (engine.hip) and the
// batched kernels (batched.hip).  Every routine reads its problem from a
// ColProblem descriptor and takes its workgroup index explicitly, so the same
// arithmetic runs in both launch schemes.
#pragma once
#include "engine.h"

#include <type_traits>

namespace {

constexpr int MAXM = 1024;  // largest m the sketch-space kernels support
constexpr int TALL_TPB = 1024;  // threads per tall workgroup

// workgroups of the float64 step of column j (FIN_P values of p each)
constexpr int FIN_P = 16;
__host__ __device__ inline int fin_groups(int32_t j) { return j > 0 ? (j + FIN_P - 1) / FIN_P : 1; }

// ------------------------------------------------------ deferred c_{j-1}
// The last coefficient of c_j = T_{j-1}^t S_{j-1}^t z_j is
//     c_{j-1} = beta_{j-1} (e_{j-1} - sum_{p < j-1} d_p c_p)
// (d = S^t s_{j-1}, e = S^t z_j).  The step of column j-1 leaves beta and e_{j-1}
// in fs[0..1] and per-workgroup partial sums of d_p c_p in dcpart[0..gfin); the
// consumers (the next reduction and tall pass) finish it themselves, so the
// step needs no cross-workgroup hand-off.  In two halves: the loads, issued
// with a kernel's first loads, and the wave sum where the value is needed
// (called by whole waves; fixed order).  gfin <= 64: one partial sum per lane.
static_assert((MAXM + FIN_P - 1) / FIN_P <= 64, "one partial sum per lane");
struct DeferredC {
  double part, f0, f1;
};
__device__ __forceinline__ DeferredC deferred_c_load(const double *__restrict__ fs,
                                                     const double *__restrict__ dcpart, int gfin) {
  const int lane = threadIdx.x & 63;
  return DeferredC{lane < gfin ? dcpart[lane] : 0.0, fs[0], fs[1]};
}
__device__ __forceinline__ double deferred_c_finish(const DeferredC &d) {
  return d.f0 * (d.f1 - wave_sum(d.part));
}

// ------------------------------------------------------------------ k_tall
// One workgroup per TILE rows; thread t owns rows base + VEC*(t + 256 v) + e.
// FAST: every 16-byte vector of the tile is in bounds and aligned; head rows
// (i < m) are loaded with the vector but excluded from the update by value, so
// they keep their input values (head rows of W are refreshed in float64 from
// U_1 = S_{1:m} by the reduction kernel).  !FAST: guarded element accesses
// (ragged last tile or unaligned storage).
// NTU: the stored columns are read with non-temporal loads (passes that apply
// more than TALL_CACHED_COLS columns stream far more than the caches hold);
// otherwise with ordinary loads (the blocked schedule's passes, whose few
// columns were written moments before and are read again by the next pass).
constexpr int TALL_CACHED_COLS = 32;
template <typename ST, bool FAST, int NV, int TPB, bool NTU, bool PRE = false, typename CP>
__device__ __forceinline__ void tall_body(ST *__restrict__ W, int64_t ldw, int64_t n, int32_t m,
                                          int32_t j, int32_t p0, bool prev,
                                          const double *__restrict__ cf, const CP &cprev_of,
                                          double iaprev, int64_t base,
                                          typename CompT<ST>::type (&acc)[NV][16 / sizeof(ST)]) {
  using CT = typename CompT<ST>::type;
  constexpr int VEC = 16 / sizeof(ST);
  const int tid = threadIdx.x;
  auto row = [&](int v) { return base + (int64_t)VEC * (tid + TPB * v); };
  auto ok = [&](int64_t i) { return i >= m && i < n; };
  const bool head = base < m;  // uniform: the tile holds head rows

  uint32_t off[NV];
#pragma unroll
  for (int v = 0; v < NV; ++v) off[v] = (uint32_t)((row(v) - base) * (int64_t)sizeof(ST));

  // acc <- w_j (PRE: already loaded by the caller)
  const ST *wj = W + (int64_t)j * ldw;
  if constexpr (!PRE) {
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t i0 = row(v);
      if (FAST) {
        vload(wj + i0, acc[v]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[v][e] = ok(i0 + e) ? cvt_in<CT>(wj[i0 + e]) : (CT)0;
      }
    }
  }
  // acc -= U_{:, <j-1} c  (stored columns, already scaled)
  if (FAST) {
    if (!head) {
      // UF columns per step so that UF * NV 16-byte loads are in flight
      constexpr int UF = NV >= 8 ? 1 : 8 / NV;
      int p = p0;
      if constexpr (UF > 1) {
#pragma unroll 1
        for (; p + UF <= j - 1; p += UF) {
          u32x4 raw[UF][NV];
#pragma unroll
          for (int u = 0; u < UF; ++u) {
            const char *cb = (const char *)(W + (int64_t)(p + u) * ldw + base);
#pragma unroll
            for (int v = 0; v < NV; ++v)
              raw[u][v] = NTU ? vraw_nt(cb + off[v]) : *reinterpret_cast<const u32x4 *>(cb + off[v]);
          }
          __builtin_amdgcn_sched_barrier(0);
#pragma unroll
          for (int u = 0; u < UF; ++u) {
            const CT cp = (CT)cf[p + u];
#pragma unroll
            for (int v = 0; v < NV; ++v) {
              CT x[VEC];
              vdecode<ST, CT>(raw[u][v], x);
#pragma unroll
              for (int e = 0; e < VEC; ++e) acc[v][e] -= x[e] * cp;
            }
          }
        }
      }
#pragma unroll 1
      for (; p < j - 1; ++p) {
        const CT cp = (CT)cf[p];
        const char *cb = (const char *)(W + (int64_t)p * ldw + base);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          CT x[VEC];
          vload<ST, CT, NTU>((const ST *)(cb + off[v]), x);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[v][e] -= x[e] * cp;
        }
      }
    } else {
#pragma unroll 1
      for (int p = p0; p < j - 1; ++p) {
        const CT cp = (CT)cf[p];
        const char *cb = (const char *)(W + (int64_t)p * ldw + base);
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int64_t i0 = row(v);
          CT x[VEC];
          vload<ST, CT, true>((const ST *)(cb + off[v]), x);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[v][e] -= (i0 + e >= m) ? x[e] * cp : (CT)0;
        }
      }
    }
  } else {
#pragma unroll 1
    for (int p = p0; p < j - 1; ++p) {
      const CT cp = (CT)cf[p];
      const ST *col = W + (int64_t)p * ldw;
#pragma unroll
      for (int v = 0; v < NV; ++v) {
        const int64_t i0 = row(v);
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (ok(i0 + e)) acc[v][e] -= cvt_in<CT>(col[i0 + e]) * cp;
      }
    }
  }
  // previous column: raw refreshed values, used, then stored scaled by
  // 1/alpha_{j-1}.  Column 0 is never refreshed: its raw values are the input.
  // (prev == false: column j-1 was already stored scaled and applied by the
  // panel update of the blocked schedule.)
  if (j >= 1 && prev) {
    const CT cp = (CT)cprev_of();  // formed only now: its loads were issued first
    const CT ia = (CT)iaprev;
    ST *col = W + (int64_t)(j - 1) * ldw;
#pragma unroll
    for (int v = 0; v < NV; ++v) {
      const int64_t i0 = row(v);
      CT x[VEC], o[VEC];
      if (FAST) {
        vload(col + i0, x);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          if (i0 + e >= m) acc[v][e] -= x[e] * cp;
          o[e] = x[e] * ia;
        }
        vstore(col + i0, o);  // head rows are rewritten from S at the end
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          if (ok(i0 + e)) {
            x[e] = cvt_in<CT>(col[i0 + e]);
            acc[v][e] -= x[e] * cp;
            col[i0 + e] = cvt_out<ST>((double)(x[e] * ia));
          }
        }
      }
    }
  }
  // store the raw refreshed column in place (in the storage type); the first
  // pass of a panel in the blocked schedule applies nothing (the panel update
  // has), so w_j is unchanged and is not written back
  const bool applied = p0 < j - 1 || (j >= 1 && prev);  // uniform
  if (!applied) return;
  ST *wjw = W + (int64_t)j * ldw;
#pragma unroll
  for (int v = 0; v < NV; ++v) {
    const int64_t i0 = row(v);
    if (FAST) {
      vstore(wjw + i0, acc[v]);  // head rows hold their unchanged input values
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (ok(i0 + e)) wjw[i0 + e] = cvt_out<ST>((double)acc[v][e]);
    }
  }
}

// A tall workgroup covers TPW consecutive transform tiles (TPW * TILE rows),
// so the per-column partials shrink by TPW.
//
// The transform's order of butterflies depends only on the storage type and
// TPW, never on TPB, so that every launch scheme gives bitwise the same
// partials.  It is defined for the 1024-thread layout, li = VEC (t + 1024 v)
// + e (t < 1024): the low VL bits (the elements of a 16-byte vector) and the
// bits from VL + 10 up (a thread's vectors) are a thread's own, the 10 bits
// between are the thread index.  Own values are transformed in registers:
// within-tile bits and tile-index bits alike (the butterflies over the
// tile-index bits form the +/- combination of the workgroup's tiles that every
// sample takes, H_{n/TILE} restricted to them).  Two radix-16 LDS passes cover
// the thread-index bits [VL, VL + 8); the two thread-index bits above those are
// left to the sample reads: within-tile ones (the fold bits) as +/- sums of
// entries, tile-index ones as +/- sums of tiles.  Butterflies over distinct
// bits commute, so this is Alg. 1's transform up to rounding, with fewer LDS
// passes than three radix-16 passes per tile and one entry per sample instead
// of TPW where the tile bits are own.  With fewer threads (TPB = 256 or 512)
// a thread holds the values of 1024 / TPB threads of that layout and leaves
// the bits between them to the LDS passes and the sample reads as well.
// HALVES: the two halves of the rows are transformed apart (their top bit is
// then read at sample time too).
template <int VEC, int TPW, bool HALVES> struct TallBits {
  static constexpr int VL = VEC == 2 ? 1 : VEC == 4 ? 2 : 3;
  static constexpr int TOP = VL + 10;  // lowest own bit above the vector
  static constexpr int FLO = VL + 8;   // fold bits [FLO, FHI)
  static constexpr int FHI = TOP < TILE_LOG ? TOP : TILE_LOG;
  static constexpr int NF = FHI - FLO;
  static constexpr int FMASK = ((1 << FHI) - 1) & ~((1 << FLO) - 1);
  // tile-index bits held by the thread index, by the halves, in registers
  static constexpr int MTID = TOP > TILE_LOG ? ((1 << (TOP - TILE_LOG)) - 1) & (TPW - 1) : 0;
  static constexpr int MRAW = MTID | (HALVES ? (TPW >> 1) : 0);
  static constexpr int MREG = (TPW - 1) & ~MRAW;
  static constexpr int NRAW = (MRAW & 1) + ((MRAW >> 1) & 1);
  static_assert(VEC == 2 || VEC == 4 || VEC == 8, "16-byte vectors of 8, 4 or 2 byte values");
  static_assert(TPW <= 4, "at most two tile-index bits");
};

// x's bits deposited at the set bits of mask, lowest first
__host__ __device__ constexpr int deposit_bits(int x, int mask) {
  int r = 0, i = 0;
  for (int b = 0; b < 31; ++b)
    if ((mask >> b) & 1) {
      if ((x >> i) & 1) r |= 1 << b;
      ++i;
    }
  return r;
}

// One radix-16 pass over the bits [sh, sh + 4) of NT tiles from s, after an
// LDS-only barrier (global loads issued before it stay in flight).
template <typename A, int NT> __device__ __forceinline__ void tiles_pass16(A *s, int sh) {
  lds_barrier();
  for (int gg = threadIdx.x; gg < (TILE / 16) * NT; gg += blockDim.x) {
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

// TPB threads per workgroup: 1024 (one workgroup per compute unit on large
// problems) or 256 (several workgroups per compute unit, for the many small
// problems of a batch).  The result does not depend on TPB: every row is
// refreshed alone and the in-LDS transform runs the same butterflies.
template <typename ST, int KIND, int TPW, int TPB = TALL_TPB>
__device__ __forceinline__ void tall_block(const ColProblem &P, int32_t j, int32_t p0, int bid) {
  static_assert(KIND != RHQR_SKETCH_GAUSS || TPB == 1024, "the Gaussian tail assumes 1024 threads");
  ST *__restrict__ W = (ST *)P.W;
  const int64_t ldw = P.ldw, n = P.n;
  const int32_t m = P.m, l = P.l;
  const double *__restrict__ cf = P.cf;
  const double *__restrict__ ia = P.ia;
  double *__restrict__ part = P.part;
  const uint64_t *__restrict__ signs = P.signs;
  const int32_t *__restrict__ rows = P.rows;
  const double *__restrict__ om = P.omega;
  const int aligned = P.aligned;
  const int defer = P.defer && j >= 1;
  const int gfin = fin_groups(j - 1);
  const double *__restrict__ fs = P.fs;
  const double *__restrict__ dcpart = P.dcpart;
  using CT = typename CompT<ST>::type;
  constexpr int VEC = 16 / sizeof(ST);
  constexpr int ROWS = TILE * TPW;
  constexpr int NV = ROWS / (TPB * VEC);
  static_assert(NV >= 1, "tile too small for the vector width");
  __shared__ CT s[TPW * TILE_PAD];
  using WB = TallBits<VEC, TPW, false>;  // one transform of all rows
  using HB = TallBits<VEC, TPW, true>;   // the two halves apart
  static_assert(TPB == 1024 || TPB == 512 || TPB == 256, "1024 / TPB threads of the layout");
  const int64_t base = (int64_t)bid * ROWS;
  const bool fast = aligned && base + ROWS <= n;
  const bool prev = j - 1 >= p0;
  // SRHT: the workgroup's sign words and the first sample row, loaded now and
  // used after the streaming pass
  constexpr int NSW = ROWS / 64;
  __shared__ uint64_t sgn[KIND == RHQR_SKETCH_SRHT ? NSW : 1];
  uint64_t sw = 0;
  int32_t rq = 0;
  if (KIND == RHQR_SKETCH_SRHT) {
    const int64_t wi = base / 64 + threadIdx.x;
    if (threadIdx.x < NSW && wi * 64 < n) sw = signs[wi];
    if ((int)threadIdx.x < l) rq = rows[threadIdx.x];
  }
  // coefficient of the raw previous column: c_{j-1} / alpha_{j-1} (its loads
  // issued here, its sum formed when the previous column is applied)
  double iaprev = 0.0, cfprev = 0.0;
  DeferredC dc{0.0, 0.0, 0.0};
  if (j >= 1 && prev) {
    iaprev = ia[j - 1];
    if (defer)
      dc = deferred_c_load(fs, dcpart, gfin);
    else
      cfprev = cf[j - 1];
  }
  auto cprev_of = [&]() { return defer ? deferred_c_finish(dc) * iaprev : cfprev; };
  const int tid = threadIdx.x;
  // signed values of the rows li0 + e (li0 = VEC (tid + TPB v) + off, v below
  // the extent of a), transformed over the thread's own bits, into their tiles
  auto to_lds = [&](const auto &a, int off) {
    constexpr int NB = std::extent<std::remove_reference_t<decltype(a)>>::value;
    constexpr int NE = NB * VEC;
    CT t[NE];  // t[VEC v + e]
#pragma unroll
    for (int v = 0; v < NB; ++v) {
      const int li0 = VEC * (tid + TPB * v) + off;
      const int64_t i0 = base + li0;
      const uint64_t word = sgn[li0 >> 6];
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int64_t i = i0 + e;
        CT x = (i >= m && i < n) ? a[v][e] : (CT)0;
        if ((word >> (i & 63)) & 1ull) x = -x;
        t[v * VEC + e] = x;
      }
    }
    // bits of VEC v + e: the element bits, then the bits of v; with TPB <
    // 1024 the low bits of v are thread-index bits of the 1024-thread layout
    // (left out here)
    constexpr int SKIP = TPB == 1024 ? 0 : TPB == 512 ? 1 : 2;
    constexpr int VLB = WB::VL;
#pragma unroll
    for (int h = 1; h < NE; h <<= 1) {
      if (h >= (1 << VLB) && h < (1 << (VLB + SKIP))) continue;
#pragma unroll
      for (int i = 0; i < NE; ++i)
        if ((i & h) == 0) {
          const CT x = t[i], y = t[i + h];
          t[i] = x + y;
          t[i + h] = x - y;
        }
    }
#pragma unroll
    for (int v = 0; v < NB; ++v)
#pragma unroll
      for (int e = 0; e < VEC; ++e) {
        const int li = VEC * (tid + TPB * v) + off + e;
        s[(li >> TILE_LOG) * TILE_PAD + tpad(li & (TILE - 1))] = t[v * VEC + e];
      }
  };
  // SRHT, float64, full workgroups of several tiles: two halves, the first
  // half's tiles transformed while the second half's loads of w_j are in
  // flight (the same refresh arithmetic per row as the one-pass order; the
  // halves' top bit joins the sample reads instead of the registers;
  // narrower types, with one or two vectors per thread and half, measured
  // slower this way)
  constexpr bool PIPE =
      KIND == RHQR_SKETCH_SRHT && TPW >= 2 && NV % 2 == 0 && TPB == 1024 && sizeof(ST) == 8;
  bool piped = false;
  if constexpr (PIPE) {
    // only the short passes (at most TALL_CACHED_COLS stored columns, the
    // blocked schedule's): a long pass gains nothing from hiding one transform
    // and streams better in one piece
    if (fast && j - 1 - p0 <= TALL_CACHED_COLS) {
      piped = true;
      constexpr int NVH = NV / 2, ROWSH = ROWS / 2, TPH = TPW / 2;
      CT a0[NVH][VEC], a1[NVH][VEC];
      tall_body<ST, true, NVH, TPB, false>(W, ldw, n, m, j, p0, prev, cf, cprev_of, iaprev, base,
                                           a0);
      if (tid < NSW) sgn[tid] = sw;
      lds_barrier();
      to_lds(a0, 0);
      const ST *wj = W + (int64_t)j * ldw + base + ROWSH;
#pragma unroll
      for (int v = 0; v < NVH; ++v) vload(wj + VEC * (tid + TPB * v), a1[v]);
      tiles_pass16<CT, TPH>(s, HB::VL);
      tiles_pass16<CT, TPH>(s, HB::VL + 4);
      tall_body<ST, true, NVH, TPB, false, true>(W, ldw, n, m, j, p0, prev, cf, cprev_of, iaprev,
                                                 base + ROWSH, a1);
      to_lds(a1, ROWSH);
      tiles_pass16<CT, TPH>(s + TPH * TILE_PAD, HB::VL);
      tiles_pass16<CT, TPH>(s + TPH * TILE_PAD, HB::VL + 4);
    }
  }
  if (!piped) {
    CT acc[NV][VEC];
    if (fast && j - 1 - p0 > TALL_CACHED_COLS)
      tall_body<ST, true, NV, TPB, true>(W, ldw, n, m, j, p0, prev, cf, cprev_of, iaprev, base,
                                         acc);
    else if (fast)
      tall_body<ST, true, NV, TPB, false>(W, ldw, n, m, j, p0, prev, cf, cprev_of, iaprev, base,
                                          acc);
    else
      tall_body<ST, false, NV, TPB, false>(W, ldw, n, m, j, p0, prev, cf, cprev_of, iaprev, base,
                                           acc);
    if (KIND == RHQR_SKETCH_IDENT) return;
    if (KIND == RHQR_SKETCH_SRHT) {
      if (tid < NSW) sgn[tid] = sw;
      lds_barrier();
      to_lds(acc, 0);
      tiles_pass16<CT, TPW>(s, WB::VL);
      tiles_pass16<CT, TPW>(s, WB::VL + 4);
    } else {
      // Gaussian: partial Omega[:, rows] w~_rows, four row groups per sample
        // Each thread takes two adjacent samples (one 16-byte load of Omega per
        // row when l is even) and four accumulators over rows 16 apart, so that
        // four loads per thread are in flight; odd l (or an Omega not 16-byte
        // aligned) takes the samples one by one.
        __shared__ double red[KIND == RHQR_SKETCH_GAUSS ? 2048 : 1];
#pragma unroll
        for (int v = 0; v < NV; ++v) {
          const int li0 = VEC * (tid + TPB * v);
#pragma unroll
          for (int e = 0; e < VEC; ++e) {
            const int64_t i = base + li0 + e;
            s[li0 + e] = (i >= m && i < n) ? acc[v][e] : (CT)0;
          }
        }
        const int64_t lo = base > m ? base : (int64_t)m;
        const int64_t hi = base + ROWS < n ? base + ROWS : n;
        const int g = tid >> 8, t = tid & 255;
        const bool pairs = (l & 1) == 0 && ((uintptr_t)om & 15) == 0;
        for (int q0 = 0; q0 < l; q0 += 512) {
          __syncthreads();
          const int q = q0 + 2 * t;
          double a[4] = {0.0, 0.0, 0.0, 0.0}, b[4] = {0.0, 0.0, 0.0, 0.0};
          if (pairs && q < l) {  // q + 1 < l as well (l even, q even)
            int64_t i = lo + g;
#pragma unroll 2
            for (; i + 12 < hi; i += 16) {
#pragma unroll
              for (int u = 0; u < 4; ++u) {
                const double2 o = *reinterpret_cast<const double2 *>(om + (i + 4 * u - m) * l + q);
                const double x = (double)s[i + 4 * u - base];
                a[u] += o.x * x;
                b[u] += o.y * x;
              }
            }
            for (; i < hi; i += 4) {
              const double2 o = *reinterpret_cast<const double2 *>(om + (i - m) * l + q);
              const double x = (double)s[i - base];
              a[0] += o.x * x;
              b[0] += o.y * x;
            }
          } else if (!pairs) {
            for (int e = 0; e < 2; ++e) {
              if (q + e >= l) break;
              double c = 0.0;
              for (int64_t i = lo + g; i < hi; i += 4) c += om[(i - m) * l + q + e] * (double)s[i - base];
              (e ? b : a)[0] = c;
            }
          }
          red[2 * (g * 256 + t)] = (a[0] + a[1]) + (a[2] + a[3]);
          red[2 * (g * 256 + t) + 1] = (b[0] + b[1]) + (b[2] + b[3]);
          __syncthreads();
          if (tid < 512 && q0 + tid < l)  // sample q0 + tid of row group g is red[512 g + tid]
            part[(int64_t)bid * l + q0 + tid] =
                (red[tid] + red[512 + tid]) + (red[1024 + tid] + red[1536 + tid]);
        }
    }
  }
  if (KIND == RHQR_SKETCH_SRHT) {
    // sample q (row r = TILE r1 + r2): the tiles t0 + tt of this workgroup
    // enter with sign (-1)^popcount(r1 & (t0 + tt)) = that of r1 & t0 times
    // that of r1 & tt; the slot r1 & MREG holds the combination over the
    // register tile bits, the others are summed here
    lds_barrier();
    const uint64_t t0 = (uint64_t)bid * TPW;
    auto samples = [&](auto bits) {
      using B = decltype(bits);
      for (int q = tid; q < l; q += TPB) {
        const int32_t r = q == tid ? rq : rows[q];
        const int r2 = r & (TILE - 1);
        const uint64_t r1 = (uint64_t)(r >> TILE_LOG);
        const int rb = r2 & ~B::FMASK;
        const int treg = (int)(r1 & (uint64_t)B::MREG);
        double h = 0.0;
#pragma unroll
        for (int x = 0; x < (1 << B::NRAW); ++x) {
          const int tau = deposit_bits(x, B::MRAW);
#pragma unroll
          for (int y = 0; y < (1 << B::NF); ++y) {
            const int f = y << B::FLO;
            const double v = (double)s[(tau | treg) * TILE_PAD + tpad(rb | f)];
            const int par = __popc((unsigned)(r1 & (uint64_t)tau)) + __popc((unsigned)(r2 & f));
            h += (par & 1) ? -v : v;
          }
        }
        part[(int64_t)bid * l + q] = (__popcll(r1 & t0) & 1) ? -h : h;
      }
    };
    if (piped)
      samples(HB{});
    else
      samples(WB{});
  }
}


// ------------------------------------------------------------------- k_red
// One workgroup per RED_CHUNK rows of the (l+m) sketch space (head chunks
// first).  Forms y = Psi w~_j on its rows: head rows y_k = w_{k,j} - sum_{p<j}
// S_{k,p} c_p (float64), tail rows the sum of the per-workgroup sketch
// partials (SRHT scaled by l^-1/2), or the refreshed rows themselves for
// Psi = I.  Then, on its rows, the partial sums that RHVector and the T/c
// updates need, with y masked to rows k >= j (no cancellation against the
// already-eliminated entries):
//   sq     = sum y_k^2                       (rho^2)
//   dpart_p = sum S_{k,p} y_k      (p < j)   (S^t s_j up to the pivot term)
//   epart_p = sum S_{k,p} z_k      (p < j)   (S^t z_{j+1}, z the next pre-sketch)
//   ypart   = sum y_k z_k                    (s_j^t z_{j+1} up to the pivot term)
// Every load that does not depend on y (the S entries of the dot products, z,
// the partials) is issued before the first wait.
constexpr int RED_NP = 8;  // per-lane loads issued together

// RW waves per workgroup (16 with 1024 threads, 4 with 256).  The row sums
// are formed in 16 fixed groups (element t of a row's sum belongs to group
// t mod 16, each group summed in increasing t, then the groups in order) and
// every dot product by the same wave_sum8 tree (the same for any of its eight
// slots), so the result does not depend on RW and equals red_split_block's.
template <typename ST, int KIND, int RW = 16>
__device__ __forceinline__ void red_block(const ColProblem &P, int32_t j, int next, int bid) {
  static_assert(16 % RW == 0, "RW must divide 16");
  const ST *__restrict__ W = (const ST *)P.W;
  const int64_t ldw = P.ldw;
  const int32_t m = P.m, l = P.l;
  const double *__restrict__ Z = P.Z;
  const int64_t ldz = P.ldz;
  const double *__restrict__ S = P.S;
  const int64_t lds = P.lds;
  const double *__restrict__ c = P.c;
  const int defer = P.defer && j >= 1;
  const int gfin = fin_groups(j - 1);
  const double *__restrict__ fs = P.fs;
  const double *__restrict__ dcpart = P.dcpart;
  const double *__restrict__ part = P.part;
  const int64_t nparts = P.nparts;
  const double scale = P.scale;
  double *__restrict__ y = P.y;
  double *__restrict__ sq = P.sq;
  double *__restrict__ dpart = P.dpart;
  double *__restrict__ epart = P.epart;
  double *__restrict__ ypart = P.ypart;
  __shared__ double red[16][RED_CHUNK + 1];
  __shared__ double yl[RED_CHUNK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nhb = (m + RED_CHUNK - 1) / RED_CHUNK;
  const bool head = bid < nhb;
  const int k = head ? bid * RED_CHUNK + lane : m + (bid - nhb) * RED_CHUNK + lane;
  const bool valid = head ? (k < m) : (k < m + l);
  // S entries of the first RED_NP dot products of this wave, and z
  double sp[RED_NP];
#pragma unroll
  for (int b = 0; b < RED_NP; ++b) {
    const int p = w + RW * b;
    sp[b] = (valid && p < j) ? S[k + (int64_t)p * lds] : 0.0;
  }
  const double z = (next && valid) ? Z[k + (int64_t)(j + 1) * ldz] : 0.0;
  const DeferredC dc = (j >= 1 && head && defer) ? deferred_c_load(fs, dcpart, gfin)
                                                 : DeferredC{0.0, 0.0, 0.0};
#pragma unroll
  for (int gi = 0; gi < 16 / RW; ++gi) {
    const int g = w + RW * gi;  // this group's elements: g, g + 16, g + 32, ...
    double v = 0.0;
    if (j >= 1) {
      if (head) {
        // loads with clamped indices, issued together; terms with p >= pe
        // are zeros, as before
        const int pe = valid ? min(j, k + 1) : 0;
        const int kc = valid ? k : 0;
        for (int p0 = g; p0 < j; p0 += 16 * RED_NP) {
          double sv[RED_NP], cv[RED_NP];
#pragma unroll
          for (int b = 0; b < RED_NP; ++b) {
            const int p = min(p0 + 16 * b, j - 1);
            sv[b] = S[kc + (int64_t)p * lds];
            cv[b] = c[p];
          }
          // the deferred c_{j-1}, formed after this batch's loads are issued
          const double clast = defer ? deferred_c_finish(dc) : 0.0;
          double t[RED_NP];
#pragma unroll
          for (int b = 0; b < RED_NP; ++b) {
            const int p = p0 + 16 * b;
            const double cp = (defer && p == j - 1) ? clast : cv[b];
            t[b] = (p < pe && p >= P.c0) ? sv[b] * cp : 0.0;
          }
#pragma unroll
          for (int b = 0; b < RED_NP; ++b) v += t[b];
        }
      } else if (KIND != RHQR_SKETCH_IDENT && valid) {
        const double *pq = part + (k - m);
        for (int64_t t0 = g; t0 < nparts; t0 += 16 * RED_NP) {
          double t[RED_NP];
#pragma unroll
          for (int b = 0; b < RED_NP; ++b) {
            const int64_t tt = t0 + 16 * b;
            t[b] = tt < nparts ? pq[tt * l] : 0.0;
          }
#pragma unroll
          for (int b = 0; b < RED_NP; ++b) v += t[b];
        }
      }
    }
    red[g][lane] = v;
  }
  __syncthreads();
  if (w == 0) {
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += red[i][lane];
    double out = 0.0;
    if (valid) {
      if (j == 0)
        out = Z[k];  // column 0 of the pre-sketch
      else if (head)
        out = cvt_in<double>(W[k + (int64_t)j * ldw]) - s;
      else if (KIND == RHQR_SKETCH_IDENT)
        out = cvt_in<double>(W[k + (int64_t)j * ldw]);
      else
        out = s * scale;
      y[k] = out;
    }
    const double ym = (valid && k >= j) ? out : 0.0;
    yl[lane] = ym;
    const double tot = wave_sum(ym * ym);
    const double yz = next ? wave_sum(ym * z) : 0.0;
    if (lane == 0) {
      sq[bid] = tot;
      if (next) ypart[bid] = yz;
    }
  }
  __syncthreads();
  const double ym = yl[lane];
  // partial dot products with the earlier columns of S, one wave per p
  for (int p0 = w; p0 < j; p0 += RW * RED_NP) {
    if (p0 > w) {  // columns beyond the prefetched ones (j > RW RED_NP)
#pragma unroll
      for (int b = 0; b < RED_NP; ++b) {
        const int p = p0 + RW * b;
        sp[b] = (valid && p < j) ? S[k + (int64_t)p * lds] : 0.0;
      }
    }
#pragma unroll
    for (int b0 = 0; b0 < RED_NP; b0 += 4) {
      if (p0 + RW * b0 < j) {  // uniform across the wave
        double pr[8];
#pragma unroll
        for (int b = 0; b < 4; ++b) {
          pr[b] = sp[b0 + b] * ym;
          pr[4 + b] = next ? sp[b0 + b] * z : 0.0;
        }
        const double tot = wave_sum8(pr);
        const int idx = lane >> 3, p = p0 + RW * (b0 + (idx & 3));
        if ((lane & 7) == 0 && p < j) {
          if (idx < 4)
            dpart[(int64_t)bid * m + p] = tot;
          else if (next)
            epart[(int64_t)bid * m + p] = tot;
        }
      }
    }
  }
}

// k_red of one problem, with the dot products split over workgroups by p:
// workgroup (r, chunk) forms y on the chunk's RED_CHUNK rows exactly as
// red_block does (split 0 alone writes y, sq and ypart) and then only the
// partial sums for p in [RSP r, RSP (r + 1)), four per wave, reduced by one
// wave_sum8 per wave.  All loads that do not depend on y are issued in one
// batch (RH_NP S entries per lane of the head rows, RT_NP partial sketches per
// lane of the tail rows; more only beyond 16 RH_NP columns or 16 RT_NP tiles).
// The row sums are formed in the same 16 fixed groups as red_block.
constexpr int RSP = 64;     // values of p per workgroup (16 waves x 4)
constexpr int RH_NP = 16;   // head: S entries per lane loaded together
constexpr int RT_NP = 16;   // tail: partial sketches per lane loaded together
__host__ __device__ inline int red_splits(int32_t j) { return j > RSP ? (j + RSP - 1) / RSP : 1; }

template <typename ST, int KIND>
__device__ __forceinline__ void red_split_block(const ColProblem &P, int32_t j, int next, int bid,
                                                int split) {
  const ST *__restrict__ W = (const ST *)P.W;
  const int64_t ldw = P.ldw;
  const int32_t m = P.m, l = P.l;
  const double *__restrict__ Z = P.Z;
  const int64_t ldz = P.ldz;
  const double *__restrict__ S = P.S;
  const int64_t lds = P.lds;
  const double *__restrict__ c = P.c;
  const int defer = P.defer && j >= 1;
  const int gfin = fin_groups(j - 1);
  const double *__restrict__ fs = P.fs;
  const double *__restrict__ dcpart = P.dcpart;
  const double *__restrict__ part = P.part;
  const int64_t nparts = P.nparts;
  const double scale = P.scale;
  __shared__ double red[16][RED_CHUNK + 1];
  __shared__ double yl[RED_CHUNK];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int nhb = (m + RED_CHUNK - 1) / RED_CHUNK;
  const bool head = bid < nhb;
  const int k = head ? bid * RED_CHUNK + lane : m + (bid - nhb) * RED_CHUNK + lane;
  const bool valid = head ? (k < m) : (k < m + l);
  const int pb = split * RSP + w;  // this wave's values of p: pb + 16 b, b < 4
  double sp[4];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    const int p = pb + 16 * b;
    sp[b] = (valid && p < j) ? S[k + (int64_t)p * lds] : 0.0;
  }
  const double z = (next && valid) ? Z[k + (int64_t)(j + 1) * ldz] : 0.0;
  const bool rawrow = w == 0 && valid && j >= 1 && (head || KIND == RHQR_SKETCH_IDENT);
  const double wjk = rawrow ? cvt_in<double>(W[k + (int64_t)j * ldw]) : 0.0;
  const double z0 = (w == 0 && valid && j == 0) ? Z[k] : 0.0;
  const DeferredC dc = (j >= 1 && head && defer) ? deferred_c_load(fs, dcpart, gfin)
                                                 : DeferredC{0.0, 0.0, 0.0};
  double v = 0.0;
  if (j >= 1) {
    if (head) {
      const int pe = valid ? min(j, k + 1) : 0;
      const int kc = valid ? k : 0;
      for (int p0 = w; p0 < j; p0 += 16 * RH_NP) {
        double sv[RH_NP], cv[RH_NP];
#pragma unroll
        for (int b = 0; b < RH_NP; ++b) {
          const int p = min(p0 + 16 * b, j - 1);
          sv[b] = S[kc + (int64_t)p * lds];
          cv[b] = c[p];
        }
        // the deferred c_{j-1}, formed after this batch's loads are issued
        const double clast = defer ? deferred_c_finish(dc) : 0.0;
#pragma unroll
        for (int b = 0; b < RH_NP; ++b) {
          const int p = p0 + 16 * b;
          const double cp = (defer && p == j - 1) ? clast : cv[b];
          v += (p < pe && p >= P.c0) ? sv[b] * cp : 0.0;
        }
      }
    } else if (KIND != RHQR_SKETCH_IDENT && valid) {
      const double *pq = part + (k - m);
      for (int64_t t0 = w; t0 < nparts; t0 += 16 * RT_NP) {
        double t[RT_NP];
#pragma unroll
        for (int b = 0; b < RT_NP; ++b) {
          const int64_t tt = t0 + 16 * b;
          t[b] = tt < nparts ? pq[tt * l] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < RT_NP; ++b) v += t[b];
      }
    }
  }
  red[w][lane] = v;
  __syncthreads();
  if (w == 0) {
    double s = 0.0;
    for (int i = 0; i < 16; ++i) s += red[i][lane];
    double out = 0.0;
    if (valid) {
      if (j == 0)
        out = z0;  // column 0 of the pre-sketch
      else if (head)
        out = wjk - s;
      else if (KIND == RHQR_SKETCH_IDENT)
        out = wjk;
      else
        out = s * scale;
      if (split == 0) P.y[k] = out;
    }
    const double ym = (valid && k >= j) ? out : 0.0;
    yl[lane] = ym;
    if (split == 0) {
      const double tot = wave_sum(ym * ym);
      const double yz = next ? wave_sum(ym * z) : 0.0;
      if (lane == 0) {
        P.sq[bid] = tot;
        if (next) P.ypart[bid] = yz;
      }
    }
  }
  __syncthreads();
  if (pb >= j) return;  // uniform across the wave; no barrier follows
  const double ym = yl[lane];
  double pr[8];
#pragma unroll
  for (int b = 0; b < 4; ++b) {
    pr[b] = sp[b] * ym;
    pr[4 + b] = next ? sp[b] * z : 0.0;
  }
  const double tot = wave_sum8(pr);
  const int idx = lane >> 3, b = idx & 3, p = pb + 16 * b;
  if ((lane & 7) == 0 && p < j) {
    if (idx < 4)
      P.dpart[(int64_t)bid * m + p] = tot;
    else if (next)
      P.epart[(int64_t)bid * m + p] = tot;
  }
}

// -------------------------------------------------------------------- scalars
struct StepScalars {
  double sigma, rho, alpha, beta, gamma;
  int ident;
  int nonfinite;  // rho or the pivot entry is NaN or infinite
};

// ss: the sum of the partial sums of squares (rho^2), yj = y_j
__device__ __forceinline__ StepScalars step_scalars(double yj, double ss, int scaling) {
  StepScalars r;
  r.rho = sqrt(ss);
  r.sigma = yj >= 0.0 ? 1.0 : -1.0;
  r.nonfinite = !(isfinite(ss) && isfinite(yj));
  r.ident = !(r.rho > 0.0);
  if (r.ident) {
    r.gamma = 0.0;
    r.alpha = 1.0;
    r.beta = 0.0;
  } else {
    r.gamma = yj + r.sigma * r.rho;
    if (scaling == RHQR_SCALE_UNIT_PIVOT) {
      r.alpha = r.gamma;
      r.beta = fabs(r.gamma) / r.rho;
    } else {
      r.alpha = sqrt(r.rho * fabs(r.gamma));
      r.beta = 1.0;
    }
  }
  return r;
}

// ------------------------------------------------------------------- k_fin
// RHVector (Alg. 2) and the T / c updates of Alg. 4 for column j, float64:
//   scalars sigma, rho, gamma, alpha, beta from the partial sums of squares;
//   s_j = ((0; y_{j:}) + sigma rho e_j) / alpha  -> S_{:, j};  R_{:, j};
//   d = S^t s_j,  e = S^t z_{j+1}  (from the k_red partials plus the pivot term);
//   T_{p,j} = -beta (T_{j-1} d)_p,  c_{j+1,p} = (T_{j-1}^t e)_p  for p < j,
// one wave per p, FIN_P values of p per workgroup; T_{j,j} = beta.  The last
// coefficient c_{j+1,j} is left to its consumers (DeferredC): workgroup g
// writes sum_{p in g} d_p c_{j+1,p} to dcpart[g], workgroup 0 writes beta and
// e_j to fs.  The partial sums, the rows of T and the pivot row of S are all
// loaded before the first wait.
constexpr int FIN_NQ = 4;  // T entries per lane loaded together
constexpr int FIN_GB = 8;  // reduction groups' partial sums loaded together

__device__ __forceinline__ void fin_block(const ColProblem &P, int32_t j, int next, int bid,
                                          int nblk) {
  const int32_t m = P.m, l = P.l;
  const int scaling = P.scaling, gred = P.gred;
  const double *__restrict__ y = P.y;
  const double *__restrict__ sq = P.sq;
  const double *__restrict__ dpart = P.dpart;
  const double *__restrict__ epart = P.epart;
  const double *__restrict__ ypart = P.ypart;
  const double *__restrict__ Z = P.Z;
  const int64_t ldz = P.ldz;
  double *__restrict__ S = P.S;
  const int64_t lds = P.lds;
  double *__restrict__ T = P.T;
  const int64_t ldt = P.ldt;
  double *__restrict__ Tt = P.Tt;
  double *__restrict__ R = P.R;
  const int64_t ldr = P.ldr;
  double *__restrict__ scal = P.scal;
  double *__restrict__ c = P.c;
  double *__restrict__ cf = P.cf;
  double *__restrict__ ia = P.ia;
  int32_t *__restrict__ status = P.status;
  double *__restrict__ dcpart = P.dcpart;
  double *__restrict__ fs = P.fs;
  __shared__ double d[MAXM], e[MAXM + 1];
  __shared__ double pd[1024], pe[1024];  // per-sub partial dot products
  __shared__ double wdc[16];
  __shared__ StepScalars shs;
  __shared__ double yzs;
  const bool needc = next != 0;
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = bid * FIN_P + w;  // this wave's index (p < j)
  // ---- loads that need nothing computed here
  // this wave's row of T (T_{p,q}, q in [p, j): from the transposed copy) and
  // column of T (T_{q,p}, q <= p)
  double tr[FIN_NQ], tc[FIN_NQ];
  const bool pw = w < FIN_P && p < j;
  const int c0 = P.c0;
#pragma unroll
  for (int i = 0; i < FIN_NQ; ++i) {
    const int qr = p + lane + 64 * i, qc = lane + 64 * i;
    tr[i] = (pw && qr < j) ? Tt[qr + (int64_t)p * m] : 0.0;
    tc[i] = (pw && needc && qc <= p && qc >= c0) ? T[qc + (int64_t)p * ldt] : 0.0;
  }
  // wave 0: the first 128 groups' partial sums of squares and of y^t z, and
  // y_j; every thread: the entry of y its first row of s_j needs
  double sqv[2] = {0.0, 0.0}, ypv[2] = {0.0, 0.0}, yj = 0.0;
  if (w == 0) {
    yj = y[j];
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int g = lane + 64 * h;
      if (g < gred) {
        sqv[h] = sq[g];
        if (needc) ypv[h] = ypart[g];
      }
    }
  }
  const int kfirst = bid * blockDim.x + threadIdx.x;
  const double yfirst = kfirst > j && kfirst < l + m ? y[kfirst] : 0.0;
  // the partial dot products d_q, e_q: thread (sub, qq) with qq = t mod QW
  // (QW the power of two >= j, at least 64) adds the groups g = sub + nsub i
  // (nsub = 1024 / QW), loaded FIN_GB at a time (clamped indices, issued
  // together) in increasing i; thread q adds the nsub sums in increasing sub
  // after the barrier.  Thread q also loads the pivot-row entry S_{j,q}.
  const int q = threadIdx.x;
  const int QW = j <= 64 ? 64 : j <= 128 ? 128 : j <= 256 ? 256 : j <= 512 ? 512 : 1024;
  const int nsub = 1024 / QW, qq = q & (QW - 1), sub = q / QW;
  const double sjq = q < j ? S[j + (int64_t)q * lds] : 0.0;
  {
    double dv = 0.0, ev = 0.0;
    if (qq < j) {
      for (int g0 = sub; g0 < gred; g0 += nsub * FIN_GB) {
        double dl[FIN_GB], el[FIN_GB];
#pragma unroll
        for (int b = 0; b < FIN_GB; ++b) {
          const int g = min(g0 + nsub * b, gred - 1);
          dl[b] = dpart[(int64_t)g * m + qq];
          el[b] = needc ? epart[(int64_t)g * m + qq] : 0.0;
        }
#pragma unroll
        for (int b = 0; b < FIN_GB; ++b)
          if (g0 + nsub * b < gred) {
            dv += dl[b];
            if (needc) ev += el[b];
          }
      }
    }
    pd[q] = dv;
    pe[q] = ev;
  }
  if (w == 0) {
    double ss = 0.0, yz = 0.0;
#pragma unroll
    for (int h = 0; h < 2; ++h)
      if (lane + 64 * h < gred) {
        ss += sqv[h];
        if (needc) yz += ypv[h];
      }
    for (int g = lane + 128; g < gred; g += 64) {  // sketches of more than 7168 rows
      ss += sq[g];
      if (needc) yz += ypart[g];
    }
    ss = wave_sum(ss);
    yz = wave_sum(yz);
    if (lane == 0) {
      shs = step_scalars(yj, ss, scaling);
      yzs = yz;
    }
  }
  __syncthreads();
  const StepScalars sc = shs;
  const double sr = sc.sigma * sc.rho;
  if (q < j) {
    double dv = 0.0, ev = 0.0;
    for (int i = 0; i < nsub; ++i) {
      dv += pd[q + QW * i];
      ev += pe[q + QW * i];
    }
    d[q] = sc.ident ? sjq : (dv + sr * sjq) / sc.alpha;
    e[q] = ev;
  }
  if (q == j && needc) {
    const double zj = Z[j + (int64_t)(j + 1) * ldz];
    e[j] = sc.ident ? zj : (yzs + sr * zj) / sc.alpha;
  }
  // s_j into S_{:, j} (grid-stride over the l+m rows)
  const int L = l + m;
  for (int k = kfirst; k < L; k += nblk * blockDim.x) {
    double s = 0.0;
    if (k == j)
      s = sc.ident ? 1.0 : (scaling == RHQR_SCALE_UNIT_PIVOT ? 1.0 : sc.gamma / sc.alpha);
    else if (k > j)
      s = sc.ident ? 0.0 : (k == kfirst ? yfirst : y[k]) / sc.alpha;
    S[k + (int64_t)j * lds] = s;
  }
  __syncthreads();
  const double beta = sc.beta;
  double dcw = 0.0;
  if (pw) {
    double td = 0.0, te = 0.0;
#pragma unroll
    for (int i = 0; i < FIN_NQ; ++i) {
      const int qr = p + lane + 64 * i, qc = lane + 64 * i;
      if (qr < j) td += tr[i] * d[qr];
      if (needc && qc <= p && qc >= c0) te += tc[i] * e[qc];
    }
    // rows beyond the prefetched ones (j > 64 FIN_NQ)
    for (int qr = p + lane + 64 * FIN_NQ; qr < j; qr += 64) td += Tt[qr + (int64_t)p * m] * d[qr];
    if (needc)
      for (int qc = lane + 64 * FIN_NQ; qc <= p; qc += 64)
        if (qc >= c0) te += T[qc + (int64_t)p * ldt] * e[qc];
    td = wave_sum(td);
    te = wave_sum(te);
    dcw = d[p] * te;
    if (lane == 0) {
      const double t = -beta * td;
      T[p + (int64_t)j * ldt] = t;
      Tt[j + (int64_t)p * m] = t;
      if (needc) {
        c[p] = te;
        cf[p] = te;
      }
    }
  }
  if (lane == 0 && w < 16) wdc[w] = dcw;
  __syncthreads();
  if (threadIdx.x == 0) {
    if (needc) {
      double s = 0.0;
      for (int i = 0; i < 16; ++i) s += wdc[i];
      dcpart[bid] = s;
    }
    if (bid == 0) {
      T[j + (int64_t)j * ldt] = beta;
      Tt[j + (int64_t)j * m] = beta;
      ia[j] = sc.ident ? 0.0 : 1.0 / sc.alpha;
      if (needc) {
        fs[0] = beta;
        fs[1] = e[j];
      }
      scal[4 * j + 0] = sc.sigma;
      scal[4 * j + 1] = sc.rho;
      scal[4 * j + 2] = sc.alpha;
      scal[4 * j + 3] = sc.beta;
      if (sc.ident) atomicCAS(status, 0, j + 1);
      if (sc.nonfinite) atomicCAS(status + 1, 0, j + 1);
    }
  }
  if (bid == 0)
    for (int r = threadIdx.x; r < m; r += blockDim.x)
      R[r + (int64_t)j * ldr] = r < j ? y[r] : (r == j ? -sr : 0.0);
}


// ---------------------------------------------------------- blocked schedule
// Panels of PB columns (block form of the column loop, Alg. 5 with the compact
// form of Prop. 3.2): before the panel starting at column J is processed, the
// J earlier reflectors are applied to all of its columns at once,
//     W_{:, J:J+nb} -= U_{:, <J} C,   C = T_{<J}^t S_{<J}^t Z_{:, J:J+nb},
// which is exact because rows p < J of c_j = T^t S^t z_j only involve
// T_{<J}; inside the panel each column is refreshed with the reflectors
// J..j-1 only.  U_{:, <J} is then read once per panel instead of once per
// column.  The same holds one level down: inside an outer panel starting at
// J0, an inner panel at J needs only the reflectors J0..J-1 (rows J0..J-1 of
// its coefficients), the outer update having applied those below J0.

// G = S_{:, <J}^t Z_{:, J:J+nb} (J x nb, ld J), one wave per entry
constexpr int PG_NP = 8;  // sketch rows per lane loaded together
__device__ __forceinline__ void pgram_block(int32_t L, int32_t J, int32_t nb,
                                            const double *__restrict__ S, int64_t lds,
                                            const double *__restrict__ Z, int64_t ldz,
                                            double *__restrict__ G, int bid) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)bid * 16 + w;
  if (e >= (int64_t)J * nb) return;
  const int p = (int)(e % J), jj = (int)(e / J);
  const double *sp = S + (int64_t)p * lds;
  const double *zp = Z + (int64_t)(J + jj) * ldz;
  // k = lane, lane + 64, ... in increasing order, PG_NP of them loaded together
  // (clamped indices; the extra terms are skipped)
  double v = 0.0;
  for (int k0 = lane; k0 < L; k0 += 64 * PG_NP) {
    double sv[PG_NP], zv[PG_NP];
#pragma unroll
    for (int b = 0; b < PG_NP; ++b) {
      const int k = min(k0 + 64 * b, L - 1);
      sv[b] = sp[k];
      zv[b] = zp[k];
    }
#pragma unroll
    for (int b = 0; b < PG_NP; ++b)
      if (k0 + 64 * b < L) v += sv[b] * zv[b];
  }
  v = wave_sum(v);
  if (lane == 0) G[p + (int64_t)jj * J] = v;
}

// C = T_{<J}^t G: C_{p,jj} = sum_{q <= p} T_{q,p} G_{q,jj} for rows J0 <= p < J,
// stored row-major (row p at C + p * pw), rows padded to pw >= nb entries
// (zeros beyond nb): the pw coefficients of column p are contiguous and read
// unconditionally by the panel kernel.  One wave per entry (p, jj): lane i
// adds q = i, i + 64, ..., then one wave sum.  Called by whole waves.
constexpr int PTRI_WAVES = 4;  // waves (entries of one column jj) per workgroup
__device__ __forceinline__ void ptri_wave(int32_t J0, int32_t J, int32_t nb, int32_t pw,
                                          const double *__restrict__ T, int64_t ldt,
                                          const double *__restrict__ G, double *__restrict__ C,
                                          int p, int jj) {
  if (p < J0 || p >= J || jj >= pw) return;  // uniform across the wave
  const int lane = threadIdx.x & 63;
  double v = 0.0;
  if (jj < nb)
    for (int q = lane; q <= p; q += 64) v += T[q + (int64_t)p * ldt] * G[q + (int64_t)jj * J];
  v = wave_sum(v);
  if (lane == 0) C[(int64_t)p * pw + jj] = v;
}

// W[m:n, J:J+nb] -= U[m:n, K0:J] C_{K0:J}.  Each thread streams VEC
// consecutive rows of U (one 16- or 8-byte load per column) against all NBC
// panel columns, whose coefficients are read with uniform (scalar) loads; U
// is read exactly once.
constexpr int PANEL_TPB = 256;
// row pitch of a panel's coefficients (and the vector-unit kernel's width)
__host__ __device__ inline int panel_width(int nb) { return nb <= 8 ? 8 : nb <= 16 ? 16 : 32; }
constexpr int PANEL_KB = 8;  // columns of U whose loads are in flight together

// rows per thread: 16-byte loads, except 8-byte ones for 32-column panels of
// 4- and 8-byte types (fewer accumulator registers, more waves per SIMD)
template <typename ST, int NBC> constexpr int panel_vec() {
  return sizeof(ST) == 2 ? 4 : (NBC >= 32 ? 8 / (int)sizeof(ST) : 16 / (int)sizeof(ST));
}

template <typename ST, typename CT, int VEC>
__device__ __forceinline__ void panel_load(const ST *p, CT *x) {
  if constexpr (sizeof(ST) * VEC == 16) {
    vload<ST, CT, true>(p, x);
  } else if constexpr (sizeof(ST) == 8) {  // one float64
    x[0] = (CT)__builtin_nontemporal_load(p);
  } else if constexpr (sizeof(ST) == 4) {  // two float32
    typedef float f32x2v __attribute__((ext_vector_type(2)));
    const f32x2v f = __builtin_nontemporal_load(reinterpret_cast<const f32x2v *>(p));
    x[0] = (CT)f.x;
    x[1] = (CT)f.y;
  } else {  // 8 bytes: four 2-byte values
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    const u32x2 u = __builtin_nontemporal_load(reinterpret_cast<const u32x2 *>(p));
    const uint32_t wd[2] = {u.x, u.y};
#pragma unroll
    for (int e = 0; e < 4; ++e) {
      const unsigned short bits = (unsigned short)(wd[e >> 1] >> (16 * (e & 1)));
      if constexpr (std::is_same<ST, __half>::value)
        x[e] = (CT)__half2float(__ushort_as_half(bits));
      else
        x[e] = (CT)__uint_as_float(((uint32_t)bits) << 16);
    }
  }
}

template <typename ST, typename CT, int VEC>
__device__ __forceinline__ void panel_store(ST *p, const CT *x) {
  if constexpr (sizeof(ST) * VEC == 16) {
    vstore<ST, CT>(p, x);
  } else if constexpr (sizeof(ST) == 8) {
    *p = (double)x[0];
  } else if constexpr (sizeof(ST) == 4) {
    typedef float f32x2v __attribute__((ext_vector_type(2)));
    f32x2v f;
    f.x = (float)x[0];
    f.y = (float)x[1];
    *reinterpret_cast<f32x2v *>(p) = f;
  } else {  // 8 bytes: four 2-byte values
    typedef unsigned int u32x2 __attribute__((ext_vector_type(2)));
    u32x2 u;
    u.x = (uint32_t)enc16<ST>((float)x[0]) | ((uint32_t)enc16<ST>((float)x[1]) << 16);
    u.y = (uint32_t)enc16<ST>((float)x[2]) | ((uint32_t)enc16<ST>((float)x[3]) << 16);
    *reinterpret_cast<u32x2 *>(p) = u;
  }
}

// Output columns JO .. JO+nb-1 (JO = J for the blocked schedule, where the
// panel follows the reflectors it is updated with).
template <typename ST, int NBC>
__device__ __forceinline__ void panel_block(ST *__restrict__ W, int64_t ldw, int64_t n, int32_t m,
                                            int32_t K0, int32_t J, int32_t nb,
                                            const double *__restrict__ Ct, int aligned, int bid,
                                            int32_t JO) {
  using CT = typename CompT<ST>::type;
  constexpr int VEC = panel_vec<ST, NBC>();  // rows per thread
  const int64_t mb = m - (m % VEC);  // aligned start; head rows < m are not written
  const int64_t rb = mb + (int64_t)bid * PANEL_TPB * VEC;  // first row of the workgroup
  const int64_t r0 = rb + (int64_t)threadIdx.x * VEC;
  if (r0 >= n) return;
  // uniform: every thread's vector is in bounds and aligned
  const bool fast = aligned && rb + (int64_t)PANEL_TPB * VEC <= n;
  const uint32_t off = (uint32_t)(threadIdx.x * VEC * sizeof(ST));
  CT acc[VEC][NBC];
#pragma unroll
  for (int e = 0; e < VEC; ++e)
#pragma unroll
    for (int c = 0; c < NBC; ++c) acc[e][c] = (CT)0;
  // coefficients of column k: Ct[k * NBC + c], zero beyond nb (uniform
  // addresses: scalar loads)
  auto coef = [&](int k, int c) -> CT { return (CT)Ct[(int64_t)k * NBC + c]; };
  if (fast) {
    int k = K0;
    for (; k + PANEL_KB <= J; k += PANEL_KB) {
      CT xs[PANEL_KB][VEC];
#pragma unroll
      for (int u = 0; u < PANEL_KB; ++u) {
        const char *cb = (const char *)(W + (int64_t)(k + u) * ldw + rb);  // uniform
        panel_load<ST, CT, VEC>((const ST *)(cb + off), xs[u]);
      }
      // keep the PANEL_KB loads issued together ahead of the arithmetic (the
      // scheduler otherwise sinks each load to its first use)
      __builtin_amdgcn_sched_barrier(0);
#pragma unroll
      for (int u = 0; u < PANEL_KB; ++u)
#pragma unroll
        for (int c = 0; c < NBC; ++c) {
          const CT ck = coef(k + u, c);
#pragma unroll
          for (int e = 0; e < VEC; ++e) acc[e][c] += xs[u][e] * ck;
        }
    }
    for (; k < J; ++k) {
      const char *cb = (const char *)(W + (int64_t)k * ldw + rb);
      CT x[VEC];
      panel_load<ST, CT, VEC>((const ST *)(cb + off), x);
#pragma unroll
      for (int c = 0; c < NBC; ++c) {
        const CT ck = coef(k, c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e][c] += x[e] * ck;
      }
    }
  } else {
    for (int k = K0; k < J; ++k) {
      const ST *col = W + (int64_t)k * ldw + r0;
      CT x[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) x[e] = r0 + e < n ? cvt_in<CT>(col[e]) : (CT)0;
#pragma unroll
      for (int c = 0; c < NBC; ++c) {
        const CT ck = coef(k, c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e][c] += x[e] * ck;
      }
    }
  }
  if (fast && r0 >= m) {
    // whole-vector read-modify-write: partial stores would cost extra HBM
    // write and fetch traffic
#pragma unroll
    for (int c = 0; c < NBC; ++c) {
      if (c < nb) {  // uniform; a break here would stop the unrolling
        ST *wc = W + (int64_t)(JO + c) * ldw + r0;
        CT x[VEC];
        panel_load<ST, CT, VEC>(wc, x);
#pragma unroll
        for (int e = 0; e < VEC; ++e) x[e] -= acc[e][c];
        panel_store<ST, CT, VEC>(wc, x);
      }
    }
    return;
  }
#pragma unroll
  for (int c = 0; c < NBC; ++c) {
    if (c < nb) {
      ST *wc = W + (int64_t)(JO + c) * ldw + r0;
#pragma unroll
      for (int e = 0; e < VEC; ++e)
        if (r0 + e < n && r0 + e >= m)
          wc[e] = cvt_out<ST>((double)(cvt_in<CT>(wc[e]) - acc[e][c]));
    }
  }
}


// ------------------------------------------ panel update on matrix cores
// W[m:n, J:J+nb] -= U[m:n, K0:J] C_{K0:J} (nb <= NC, C with row pitch pw,
// zero beyond nb) on v_mfma_f64_16x16x4 (float64 storage) or
// v_mfma_f32_16x16x4 (float32 and 2-byte storage, float32 products and
// accumulation as on the vector units), transposed so that rows of W run
// along the 16 lanes of a product's j index:
//   D^t (panel columns x rows) = W_panel^t + (-C)^t U^t.
// Each lane loads 16 bytes (VEC = 2, 4 or 8 consecutive rows) of one column
// of U; element e of every lane forms one 16-row operand (rows VEC j + e).
// The accumulators start from the panel itself (same layout, 16-byte loads)
// and are stored back as they are.  A wave owns px_rg groups of 16 VEC rows;
// px_ks steps of 4 columns (U as raw 16-byte words, and -C) are loaded
// together ahead of their products.  Waves that cross row m or n take guarded
// element accesses; rows < m are never written.  Needs 16-byte aligned
// columns.
// The panel updates (NC <= 32) load one 4-column step per batch and are built
// for PX_MIN_WG workgroups per compute unit (4 waves per SIMD, accumulators
// in ordinary registers).  Measured at 2^22 rows against 4 steps per batch at
// 2-3 waves per SIMD (accumulators in AGPRs): float32 outer updates 0.64 ->
// 0.61 ms, the float32 batch's 16-column updates 3.03 -> 2.43 ms per launch,
// float64 outer updates 1.198 -> 1.185 ms.  The thin Q's 64-column tail
// product keeps 4 steps per batch in float64, where its FP64 matrix cores
// bound it (with one step: 13.3 ms against 9.8 ms at 2^22 x 256), and takes
// one in float32 (the 512-problem batch's thin Q: 15.3 ms against 18.0 ms).
template <typename ST, int NC> constexpr int px_ks() {
  return NC > 32 && sizeof(ST) == 8 ? 4 : 1;
}
constexpr int PX_MIN_WG = 4;
template <typename ST> constexpr int px_min_wg() { return PX_MIN_WG; }
constexpr int PX_WAVES = 4;   // waves per workgroup
constexpr int PX_MIN_NB = 8; // narrower panels stay on the vector units (k_panel)
// row groups of 16 VEC rows per wave: 64 rows (float64) or 128 rows
__host__ __device__ constexpr int px_rg(int es) { return es == 2 ? 1 : 2; }

template <typename ST, int NC, bool FULL>
__device__ __forceinline__ void panel_mx_wave(const ST *__restrict__ U, int64_t ldu,
                                              ST *__restrict__ P, int64_t ldp, bool zero,
                                              int64_t n, int32_t m, int32_t K0, int32_t K1,
                                              int32_t nb, int pw, const double *__restrict__ C,
                                              int64_t row0) {
  using CT = typename CompT<ST>::type;
  using Ops = PxOps<CT>;
  using acc_t = typename Ops::acc_t;
  using UT = std::conditional_t<sizeof(ST) == 8, uint64_t,
                                std::conditional_t<sizeof(ST) == 4, uint32_t, uint16_t>>;
  constexpr int VEC = 16 / sizeof(ST);
  constexpr int RG = px_rg(sizeof(ST));
  constexpr int GR = 16 * VEC;  // rows per group
  constexpr int NCT = NC / 16;
  const int lane = threadIdx.x & 63;
  const int i16 = lane & 15, kq = lane >> 4;
  // this lane's rows in group g: rv(g) + e, e < VEC
  auto rv = [&](int g) { return row0 + (int64_t)g * GR + VEC * i16; };
  // 16 bytes of a column from row r as raw words; !FULL: element by element,
  // rows >= n (and rows < m unless headok) read as zero
  auto ldraw = [&](const ST *col, int64_t r, bool headok) -> u32x4 {
    if constexpr (FULL) {
      return vraw_nt(col + r);
    } else {
      const UT *cu = reinterpret_cast<const UT *>(col);
      UT e[VEC];
#pragma unroll
      for (int q = 0; q < VEC; ++q) e[q] = (r + q < n && (headok || r + q >= m)) ? cu[r + q] : (UT)0;
      u32x4 u;
      __builtin_memcpy(&u, e, 16);
      return u;
    }
  };
  acc_t acc[RG][VEC][NCT];
  // acc[g][e][ct][t] = panel column 16 ct + di(kq, t), row rv(g) + e
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 16 * ct + Ops::di(kq, t);
        CT x[VEC];
        if (c < nb && !zero) {
          vdecode<ST, CT>(ldraw(P + (int64_t)c * ldp, rv(g), false), x);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e) x[e] = (CT)0;
        }
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[g][e][ct][t] = x[e];
      }
  constexpr int KS = px_ks<ST, NC>();
  for (int k0 = K0; k0 < K1; k0 += 4 * KS) {
    u32x4 ub[KS][RG];
    CT cf[KS][NCT];
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      const int k = k0 + 4 * s + kq;
      const bool kv = k < K1;
      const int kc = kv ? k : K1 - 1;  // clamped: every load is in bounds
      const ST *col = U + (int64_t)kc * ldu;
#pragma unroll
      for (int g = 0; g < RG; ++g) ub[s][g] = ldraw(col, rv(g), true);
#pragma unroll
      for (int ct = 0; ct < NCT; ++ct) {
        const int c = 16 * ct + i16;  // < NC <= pw
        const double cv = C[(int64_t)kc * pw + c];
        cf[s][ct] = (kv && c < nb) ? (CT)(-cv) : (CT)0;
      }
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int s = 0; s < KS; ++s) {
      // a column beyond J contributes zero coefficients; its (clamped) values
      // are zeroed too, so no non-finite entry can enter the sum
      const bool kv = k0 + 4 * s + kq < K1;
#pragma unroll
      for (int g = 0; g < RG; ++g) {
        CT x[VEC];
        vdecode<ST, CT>(ub[s][g], x);
#pragma unroll
        for (int e = 0; e < VEC; ++e) {
          const CT b = kv ? x[e] : (CT)0;
#pragma unroll
          for (int ct = 0; ct < NCT; ++ct) acc[g][e][ct] = Ops::mma(cf[s][ct], b, acc[g][e][ct]);
        }
      }
    }
  }
#pragma unroll
  for (int g = 0; g < RG; ++g)
#pragma unroll
    for (int ct = 0; ct < NCT; ++ct)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int c = 16 * ct + Ops::di(kq, t);
        if (c >= nb) continue;
        ST *col = P + (int64_t)c * ldp;
        const int64_t r = rv(g);
        CT v[VEC];
#pragma unroll
        for (int e = 0; e < VEC; ++e) v[e] = acc[g][e][ct][t];
        if constexpr (FULL) {
          vstore<ST, CT>(col + r, v);
        } else {
#pragma unroll
          for (int e = 0; e < VEC; ++e)
            if (r + e >= m && r + e < n) col[r + e] = cvt_out<ST>((double)v[e]);
        }
      }
}

// one workgroup of PX_WAVES waves; wave w of workgroup bid owns the rows from
// (m rounded down to VEC) + (PX_WAVES bid + w) px_rg 16 VEC.  FULL waves need
// 16-byte aligned columns of U and P.
template <typename ST, int NC>
__device__ __forceinline__ void panel_mx_block(const ST *__restrict__ U, int64_t ldu,
                                               ST *__restrict__ P, int64_t ldp, bool zero,
                                               int64_t n, int32_t m, int32_t K0, int32_t K1,
                                               int32_t nb, int pw, const double *__restrict__ C,
                                               int64_t bid) {
  constexpr int VEC = 16 / sizeof(ST);
  const int w = threadIdx.x >> 6;
  const int64_t rb = m - (m % VEC);
  constexpr int WR = px_rg(sizeof(ST)) * 16 * VEC;  // rows per wave
  const int64_t row0 = rb + (bid * PX_WAVES + w) * WR;
  if (row0 >= n) return;  // whole wave beyond the last row (uniform)
  if (row0 >= m && row0 + WR <= n)
    panel_mx_wave<ST, NC, true>(U, ldu, P, ldp, zero, n, m, K0, K1, nb, pw, C, row0);
  else
    panel_mx_wave<ST, NC, false>(U, ldu, P, ldp, zero, n, m, K0, K1, nb, pw, C, row0);
}

// workgroups of panel_mx_block over rows m..n
__host__ __device__ inline int64_t panel_mx_groups(int64_t n, int32_t m, int es) {
  const int vec = 16 / es;
  const int64_t wr = px_rg(es) * 16 * vec;
  const int64_t waves = (n - (m - m % vec) + wr - 1) / wr;
  return (waves + PX_WAVES - 1) / PX_WAVES;
}


}  // namespace
