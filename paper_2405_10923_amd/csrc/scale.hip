// Column scaling around low-precision storage (mixed-precision setting of
// Sec. 8): unit max-norm columns before rounding W to the storage type, and
// R scaled back afterwards.
#include "common.h"

namespace {

constexpr int CS_TPB = 1024;

// one workgroup per column: d_j = max_i |W_ij| over the n rows (1 if zero)
__global__ void __launch_bounds__(CS_TPB) k_colmax(int64_t n, const double *__restrict__ W,
                                                   int64_t ldw, double *__restrict__ d) {
  const double *col = W + (int64_t)blockIdx.x * ldw;
  double v = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += CS_TPB) v = fmax(v, fabs(col[i]));
  __shared__ double red[CS_TPB / 64];
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o));
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = v;
  __syncthreads();
  if (threadIdx.x == 0) {
    double mx = 0.0;
    for (int w = 0; w < CS_TPB / 64; ++w) mx = fmax(mx, red[w]);
    d[blockIdx.x] = mx > 0.0 ? mx : 1.0;
  }
}

template <typename ST> __device__ __forceinline__ ST round_to(double x);
template <> __device__ __forceinline__ double round_to<double>(double x) { return x; }
template <> __device__ __forceinline__ float round_to<float>(double x) { return (float)x; }
// 2-byte types: round to float32, then to the 2-byte type (both to nearest
// even).  The empty asm keeps the compiler from merging the two roundings
// into one direct conversion, which can differ in the last bit.
__device__ __forceinline__ float round_f32(double x) {
  float f = (float)x;
  asm volatile("" : "+v"(f));
  return f;
}
template <> __device__ __forceinline__ __half round_to<__half>(double x) {
  return __float2half_rn(round_f32(x));
}
template <> __device__ __forceinline__ __hip_bfloat16 round_to<__hip_bfloat16>(double x) {
  return __float2bfloat16(round_f32(x));
}

// Wout = W D^-1 in the storage type; grid (row blocks, m)
template <typename ST>
__global__ void __launch_bounds__(256) k_colscale(int64_t n, const double *__restrict__ W,
                                                  int64_t ldw, ST *__restrict__ Wo, int64_t ldo,
                                                  const double *__restrict__ d) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i >= n) return;
  Wo[i + (int64_t)j * ldo] = round_to<ST>(W[i + (int64_t)j * ldw] / d[j]);
}

__global__ void k_scale_r(int32_t m, double *__restrict__ R, int64_t ldr,
                          const double *__restrict__ d) {
  const int i = blockIdx.x * 256 + threadIdx.x;
  const int j = blockIdx.y;
  if (i < m) R[i + (int64_t)j * ldr] *= d[j];
}

template <typename ST>
int colscale_typed(int64_t n, int32_t m, const double *W, int64_t ldw, ST *Wo, int64_t ldo,
                   double *d, hipStream_t st) {
  hipLaunchKernelGGL(k_colmax, dim3(m), dim3(CS_TPB), 0, st, n, W, ldw, d);
  RHQR_HIP(hipGetLastError());
  const dim3 grid((unsigned)((n + 255) / 256), m);
  hipLaunchKernelGGL((k_colscale<ST>), grid, dim3(256), 0, st, n, W, ldw, Wo, ldo,
                     (const double *)d);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

}  // namespace

extern "C" int rhqr_colscale(int dtype, int64_t n, int32_t m, const double *d_W64, int64_t ldw,
                             void *d_Wout, int64_t ldo, double *d_scale, void *stream) {
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -1;
  if (n < 1 || n > ((int64_t)1 << 40)) return -2;
  if (m < 1 || m > 65535) return -3;
  if (!d_W64) return -4;
  if (ldw < n) return -5;
  if (!d_Wout) return -6;
  if (ldo < n) return -7;
  if (!d_scale) return -8;
  hipStream_t st = (hipStream_t)stream;
  switch (dtype) {
    case RHQR_F64: return colscale_typed<double>(n, m, d_W64, ldw, (double *)d_Wout, ldo, d_scale, st);
    case RHQR_F32: return colscale_typed<float>(n, m, d_W64, ldw, (float *)d_Wout, ldo, d_scale, st);
    case RHQR_F16: return colscale_typed<__half>(n, m, d_W64, ldw, (__half *)d_Wout, ldo, d_scale, st);
    case RHQR_BF16:
      return colscale_typed<__hip_bfloat16>(n, m, d_W64, ldw, (__hip_bfloat16 *)d_Wout, ldo,
                                            d_scale, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

extern "C" int rhqr_scale_r(int32_t m, double *d_R, int64_t ldr, const double *d_scale,
                            void *stream) {
  if (m < 1 || m > 65535) return -1;
  if (!d_R) return -2;
  if (ldr < m) return -3;
  if (!d_scale) return -4;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_scale_r, dim3((m + 255) / 256, m), dim3(256), 0, st, m, d_R, ldr, d_scale);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}
