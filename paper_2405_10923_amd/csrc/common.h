// Shared definitions of the gfx950 RHQR library (device helpers, handle layout).
#pragma once
#include <hip/hip_runtime.h>
#include <hip/hip_ext.h>
#include <hip/hip_fp16.h>
#include <hip/hip_bf16.h>
#include <stdint.h>
#include <stddef.h>

#include <type_traits>

#include "../../include/rhqr.h"

#define RHQR_HIP(x)                                   \
  do {                                                \
    hipError_t e_ = (x);                              \
    if (e_ != hipSuccess) return RHQR_ERR_HIP;        \
  } while (0)

// Per-kernel timing (rhqr_profile_begin / rhqr_profile_end).  While profiling
// is on, prof_events hands out a start and a stop event for one launch of
// kernel class `cls` (RHQR_PROF_*), which the dispatch itself records
// (hipExtLaunchKernel), so the time measured is the kernel's own; otherwise it
// returns null events and the launch is an ordinary one.
int prof_events(int cls, hipEvent_t *e0, hipEvent_t *e1);

// launch K, timed as class `cls` when profiling is on; returns RHQR_ERR_HIP
// from the enclosing function if the launch fails
#define RHQR_LAUNCH(cls, K, grid, block, shm, st, ...)                         \
  do {                                                                        \
    hipEvent_t e0_ = nullptr, e1_ = nullptr;                                  \
    if (prof_events((cls), &e0_, &e1_)) return RHQR_ERR_HIP;                  \
    if (e0_)                                                                  \
      hipExtLaunchKernelGGL(K, grid, block, shm, st, e0_, e1_, 0, __VA_ARGS__); \
    else                                                                      \
      hipLaunchKernelGGL(K, grid, block, shm, st, __VA_ARGS__);                \
    RHQR_HIP(hipGetLastError());                                              \
  } while (0)

// Internal sketch kind: Psi = I (used for the sketch-space Householder QR of
// recRHQR, where the "n-row" matrix is the (l+m) x m sketch itself).
enum { RHQR_SKETCH_IDENT = 2 };

// Walsh-Hadamard tile: the SRHT of R^N is split as H_N = H_{N/TILE} (x) H_TILE;
// a workgroup transforms one aligned block of TILE coordinates in LDS and only
// the l sampled outputs leave the workgroup.
constexpr int TILE_LOG = 12;
constexpr int TILE = 1 << TILE_LOG;
constexpr int TILE_PAD = TILE + TILE / 16;  // one pad slot per 16 entries
__device__ __forceinline__ int tpad(int i) { return i + (i >> 4); }

// Workgroup barrier that orders LDS accesses only: global loads issued before
// it stay in flight (a full __syncthreads waits for them).
__device__ __forceinline__ void lds_barrier() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
  __builtin_amdgcn_s_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

struct rhqr_sketch_s {
  int kind;
  int64_t n;
  int32_t m;
  int32_t l;
  uint64_t seed;
  int64_t N;          // 2^ceil(log2 n)
  uint64_t *d_signs;  // ceil(N/64) words (SRHT)
  int32_t *d_rows;    // l sampled rows, increasing (SRHT)
  double *d_omega;    // l x (n-m), ld = l (GAUSS)
  int device;
};

// ---------------------------------------------------------------- dtypes
template <typename ST> struct CompT { using type = float; };
template <> struct CompT<double> { using type = double; };

template <typename CT> __device__ __forceinline__ CT cvt_in(double x) { return (CT)x; }
template <typename CT> __device__ __forceinline__ CT cvt_in(float x) { return (CT)x; }
template <typename CT> __device__ __forceinline__ CT cvt_in(__half x) { return (CT)__half2float(x); }
template <typename CT> __device__ __forceinline__ CT cvt_in(__hip_bfloat16 x) { return (CT)__bfloat162float(x); }

template <typename ST> __device__ __forceinline__ ST cvt_out(double x);
template <> __device__ __forceinline__ double cvt_out<double>(double x) { return x; }
template <> __device__ __forceinline__ float cvt_out<float>(double x) { return (float)x; }
template <> __device__ __forceinline__ __half cvt_out<__half>(double x) { return __float2half((float)x); }
template <> __device__ __forceinline__ __hip_bfloat16 cvt_out<__hip_bfloat16>(double x) { return __float2bfloat16((float)x); }

inline size_t dtype_size(int dt) {
  switch (dt) {
    case RHQR_F64: return 8;
    case RHQR_F32: return 4;
    case RHQR_F16: return 2;
    case RHQR_BF16: return 2;
  }
  return 0;
}

inline size_t align_up(size_t x, size_t a = 256) { return (x + a - 1) / a * a; }

// -------------------------------------------------------------- 16-byte I/O
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

typedef double f64x2 __attribute__((ext_vector_type(2)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// Raw 16-byte non-temporal load and its decoding, for loops that issue a batch
// of loads before converting any of them.
__device__ __forceinline__ u32x4 vraw_nt(const void *p) {
  return __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
}
template <typename ST, typename CT>
__device__ __forceinline__ void vdecode(const u32x4 u, CT *o) {
  // (the whole vector reinterpreted at once: rebuilding each value from its
  // two words let the compiler re-load the first one with a narrower load of
  // the same address)
  if constexpr (sizeof(ST) == 8) {
    const f64x2 d = __builtin_bit_cast(f64x2, u);
    o[0] = (CT)d.x;
    o[1] = (CT)d.y;
  } else if constexpr (sizeof(ST) == 4) {
    const f32x4 f = __builtin_bit_cast(f32x4, u);
    o[0] = (CT)f.x;
    o[1] = (CT)f.y;
    o[2] = (CT)f.z;
    o[3] = (CT)f.w;
  } else {
    const uint32_t w[4] = {u.x, u.y, u.z, u.w};
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      const unsigned short b = (unsigned short)(w[k >> 1] >> (16 * (k & 1)));
      if constexpr (std::is_same<ST, __half>::value)
        o[k] = (CT)__half2float(__ushort_as_half(b));
      else
        o[k] = (CT)__uint_as_float(((uint32_t)b) << 16);
    }
  }
}

// 16-byte load decoded to CT; NT selects a non-temporal (streaming) load.
template <typename ST, typename CT, bool NT = false>
__device__ __forceinline__ void vload(const ST *p, CT *o) {
  if constexpr (sizeof(ST) == 8) {
    f64x2 d;
    if constexpr (NT)
      d = __builtin_nontemporal_load(reinterpret_cast<const f64x2 *>(p));
    else
      d = *reinterpret_cast<const f64x2 *>(p);
    o[0] = (CT)d.x;
    o[1] = (CT)d.y;
    return;
  } else if constexpr (std::is_same<ST, float>::value) {
    f32x4 f;
    if constexpr (NT)
      f = __builtin_nontemporal_load(reinterpret_cast<const f32x4 *>(p));
    else
      f = *reinterpret_cast<const f32x4 *>(p);
    o[0] = (CT)f.x;
    o[1] = (CT)f.y;
    o[2] = (CT)f.z;
    o[3] = (CT)f.w;
    return;
  }
  u32x4 uv;  // 2-byte storage
  if constexpr (NT)
    uv = __builtin_nontemporal_load(reinterpret_cast<const u32x4 *>(p));
  else
    uv = *reinterpret_cast<const u32x4 *>(p);
  vdecode<ST, CT>(uv, o);
}

template <typename ST> __device__ __forceinline__ unsigned short enc16(float v) {
  if constexpr (std::is_same<ST, __half>::value)
    return __half_as_ushort(__float2half(v));
  else
    return __bfloat16_as_ushort(__float2bfloat16(v));
}

template <typename ST, typename CT>
__device__ __forceinline__ void vstore(ST *p, const CT *v) {
  uint4 u;
  if constexpr (sizeof(ST) == 8) {
    const double a = (double)v[0], b = (double)v[1];
    u.x = (uint32_t)__double2loint(a);
    u.y = (uint32_t)__double2hiint(a);
    u.z = (uint32_t)__double2loint(b);
    u.w = (uint32_t)__double2hiint(b);
  } else if constexpr (sizeof(ST) == 4) {
    u.x = __float_as_uint((float)v[0]);
    u.y = __float_as_uint((float)v[1]);
    u.z = __float_as_uint((float)v[2]);
    u.w = __float_as_uint((float)v[3]);
  } else {
    uint32_t w[4];
#pragma unroll
    for (int k = 0; k < 4; ++k)
      w[k] = (uint32_t)enc16<ST>((float)v[2 * k]) | ((uint32_t)enc16<ST>((float)v[2 * k + 1]) << 16);
    u.x = w[0];
    u.y = w[1];
    u.z = w[2];
    u.w = w[3];
  }
  *reinterpret_cast<uint4 *>(p) = u;
}

// ---------------------------------------------------------------- reductions
// Wavefront sum with DPP row moves (butterflies inside each 16-lane row) and
// four lane reads across the rows; every lane receives the same total, summed
// in a fixed order.  All 64 lanes must be active.
template <int CTRL> __device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
template <int CTRL> __device__ __forceinline__ double dpp_mov(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xf, 0xf, false);
  return __hiloint2double(hi, lo);
}
__device__ __forceinline__ float lane_read(float v, int lane) {
  return __int_as_float(__builtin_amdgcn_readlane(__float_as_int(v), lane));
}
__device__ __forceinline__ double lane_read(double v, int lane) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), lane);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), lane);
  return __hiloint2double(hi, lo);
}
template <typename T> __device__ __forceinline__ T wave_sum(T v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x141>(v);  // row_half_mirror
  v += dpp_mov<0x140>(v);  // row_mirror: every lane holds its row's sum
  return (lane_read(v, 0) + lane_read(v, 16)) + (lane_read(v, 32) + lane_read(v, 48));
}

// Sums eight values per lane over the 64 lanes at once: each exchange across
// 32, 16 and 8 lanes keeps half of the values (own plus partner's), then the
// last eight-lane groups are summed with row moves.  Lane L returns the total
// of v[(L >> 3) & 7] (bit 5 of L selects the upper four values, bit 4 the
// upper two of those, bit 3 the second).  Fixed order: deterministic.  All 64
// lanes must be active.
__device__ __forceinline__ double wave_sum8(const double (&v)[8]) {
  const int lane = threadIdx.x & 63;
  const bool h5 = lane & 32, h4 = lane & 16, h3 = lane & 8;
  double a[4], b[2];
#pragma unroll
  for (int i = 0; i < 4; ++i)
    a[i] = (h5 ? v[i + 4] : v[i]) + __shfl_xor(h5 ? v[i] : v[i + 4], 32, 64);
#pragma unroll
  for (int i = 0; i < 2; ++i)
    b[i] = (h4 ? a[i + 2] : a[i]) + __shfl_xor(h4 ? a[i] : a[i + 2], 16, 64);
  double s = (h3 ? b[1] : b[0]) + __shfl_xor(h3 ? b[0] : b[1], 8, 64);
  s += dpp_mov<0xB1>(s);   // quad_perm [1,0,3,2]
  s += dpp_mov<0x4E>(s);   // quad_perm [2,3,0,1]
  s += dpp_mov<0x141>(s);  // row_half_mirror: the other quad of the eight lanes
  return s;
}

// Sum over a workgroup; `red` is LDS scratch of >= blockDim.x/64 entries.
// Every thread returns the total.  Fixed order: deterministic.
template <typename T> __device__ T block_sum(T v, T *red) {
  v = wave_sum(v);
  const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, nw = blockDim.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  T s = 0;
  for (int i = 0; i < nw; ++i) s += red[i];
  return s;
}

// ------------------------------------------------------- matrix-core tiles
// 16 x 16 x 4 products on matrix cores in the computation type CT
// (v_mfma_f64_16x16x4 or v_mfma_f32_16x16x4).  Operands: lane l holds
// A[i = l % 16][k = l / 16] and B[k = l / 16][j = l % 16]; the accumulator's
// element t of lane l holds D[di(l / 16, t)][l % 16] (probed: float64
// i = q + 4 t, float32 i = 4 q + t).
typedef double f64x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
template <typename CT> struct PxOps;
template <> struct PxOps<double> {
  typedef f64x4_t acc_t;
  static __device__ __forceinline__ acc_t mma(double a, double b, acc_t c) {
    return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
  }
  static constexpr __device__ int di(int q, int t) { return q + 4 * t; }
};
template <> struct PxOps<float> {
  typedef f32x4_t acc_t;
  static __device__ __forceinline__ acc_t mma(float a, float b, acc_t c) {
    return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
  }
  static constexpr __device__ int di(int q, int t) { return 4 * q + t; }
};

// General form: P[m:n, 0:nb] = (zero ? 0 : P[m:n, 0:nb]) - U[m:n, K0:K1] C_{K0:K1}
// (U and P may be columns of one array that do not overlap).

// ---------------------------------------------------------------- FWHT
// In-place unnormalised Walsh-Hadamard transform (natural order) of 16
// values: the radix-16 step of the tile transforms, which run it over groups
// of 16 entries of a tile in LDS (4 index bits per pass).
template <typename A> __device__ __forceinline__ void fwht16(A v[16]) {
#pragma unroll
  for (int h = 1; h < 16; h <<= 1) {
#pragma unroll
    for (int k = 0; k < 16; ++k) {
      if ((k & h) == 0) {
        A a = v[k], b = v[k + h];
        v[k] = a + b;
        v[k + h] = a - b;
      }
    }
  }
}

// ---------------------------------------------------------------- host side
int sketch_tail_partials_size(const rhqr_sketch_s *h, int32_t k, int *gt_out, size_t *bytes_out);
int launch_sketch(const rhqr_sketch_s *h, int dtype, int64_t n, int32_t k, const void *X,
                  int64_t ldx, double *Y, int64_t ldy, void *ws, size_t ws_bytes,
                  hipStream_t st);
size_t sketch_ws_bytes(const rhqr_sketch_s *h, int32_t k);
