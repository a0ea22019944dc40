// recRHQR (Alg. 6): RHQR reconstructed from the Householder QR of the sketch.
//
//   Z = Psi W                                  (one multi-column sketch pass)
//   S, T, R = HouseholderQR(Z)                 (float64, on the device: the
//                                               column engine run with Psi = I)
//   M = ut(T^t S^t Z)   (= -T U_1^t R, Sec. 3.3)
//   U_2 M = W_2         (blocked forward substitution, launch_trsm_blocked)
//   U = [S_{1:m}; U_2],  Q = [I; 0] - U T U_1^t (optional)
// Mode RCHOL: Q = W R^-1 with the same substitution kernel.
#include "engine.h"

#include <algorithm>
#include <cmath>

namespace {

// G = S^t Z (m x m), one wave per entry.
__global__ void __launch_bounds__(1024) k_gram(int32_t m, int32_t L, const double *__restrict__ S,
                                               int64_t lds, const double *__restrict__ Z,
                                               int64_t ldz, double *__restrict__ G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t e = (int64_t)blockIdx.x * 16 + w;
  if (e >= (int64_t)m * m) return;
  const int p = (int)(e % m), q = (int)(e / m);
  double v = 0.0;
  for (int k = lane; k < L; k += 64) v += S[k + (int64_t)p * lds] * Z[k + (int64_t)q * ldz];
  v = wave_sum(v);
  if (lane == 0) G[p + (int64_t)q * m] = v;
}

// M = ut(T^t G): M_{p,q} = sum_{r <= p} T_{r,p} G_{r,q} for p <= q, 0 below.
__global__ void k_ttg(int32_t m, const double *__restrict__ T, int64_t ldt,
                      const double *__restrict__ G, double *__restrict__ M) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int q = blockIdx.y;
  if (p >= m) return;
  double v = 0.0;
  if (p <= q)
    for (int r = 0; r <= p; ++r) v += T[r + (int64_t)p * ldt] * G[r + (int64_t)q * m];
  M[p + (int64_t)q * m] = v;
}

template <typename ST>
__global__ void k_head_copy(ST *U, int64_t ldu, int32_t m, const double *S, int64_t lds) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k < m) U[k + (int64_t)c * ldu] = cvt_out<ST>(S[k + (int64_t)c * lds]);
}

int launch_head_copy(int dtype, void *U, int64_t ldu, int32_t m, const double *S, int64_t lds,
                     hipStream_t st) {
  dim3 grid((m + 255) / 256, m);
  switch (dtype) {
    case RHQR_F64: hipLaunchKernelGGL((k_head_copy<double>), grid, dim3(256), 0, st, (double *)U, ldu, m, S, lds); break;
    case RHQR_F32: hipLaunchKernelGGL((k_head_copy<float>), grid, dim3(256), 0, st, (float *)U, ldu, m, S, lds); break;
    case RHQR_F16: hipLaunchKernelGGL((k_head_copy<__half>), grid, dim3(256), 0, st, (__half *)U, ldu, m, S, lds); break;
    case RHQR_BF16:
      hipLaunchKernelGGL((k_head_copy<__hip_bfloat16>), grid, dim3(256), 0, st, (__hip_bfloat16 *)U, ldu, m, S, lds);
      break;
    default: return RHQR_ERR_UNSUPPORTED;
  }
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

struct RecWs {
  LoopWs loop;
  double *Z, *Zc, *G, *M, *Mq, *coef;
  float *stage;  // float32 copy of the solved columns (2-byte storage)
  void *qmf;     // split coefficients of the matrix-core thin Q
  void *skws;
  size_t skws_bytes;
};

size_t rec_ws_bytes(const rhqr_sketch_s *h, int dtype, int32_t m) {
  const int32_t L = h->l + m;
  size_t b = align_up(loop_ws_bytes(RHQR_SKETCH_IDENT, RHQR_F64, L, m, h->l));
  b += 2 * align_up(sizeof(double) * (size_t)L * m);
  b += 3 * align_up(sizeof(double) * (size_t)m * m);
  b += align_up(sketch_ws_bytes(h, m));
  b += trsm_coef_bytes(m);
  b += trsm_stage_bytes(dtype, h->n, m);
  b += thin_q_bytes(m);
  return b;
}

int rec_ws_carve(const rhqr_sketch_s *h, int dtype, int32_t m, void *ws, size_t bytes, RecWs *o) {
  if (bytes < rec_ws_bytes(h, dtype, m)) return RHQR_ERR_WORKSPACE;
  const int32_t L = h->l + m;
  const size_t lb = align_up(loop_ws_bytes(RHQR_SKETCH_IDENT, RHQR_F64, L, m, h->l));
  int rc = loop_ws_carve(ws, lb, RHQR_SKETCH_IDENT, RHQR_F64, L, m, h->l, &o->loop);
  if (rc) return rc;
  char *p = (char *)ws + lb;
  auto take = [&](size_t b) {
    char *r = p;
    p += align_up(b);
    return (void *)r;
  };
  o->Z = (double *)take(sizeof(double) * (size_t)L * m);
  o->Zc = (double *)take(sizeof(double) * (size_t)L * m);
  o->G = (double *)take(sizeof(double) * (size_t)m * m);
  o->M = (double *)take(sizeof(double) * (size_t)m * m);
  o->Mq = (double *)take(sizeof(double) * (size_t)m * m);
  o->skws_bytes = align_up(sketch_ws_bytes(h, m));
  o->skws = take(o->skws_bytes);
  o->coef = (double *)take(trsm_coef_bytes(m));
  const size_t sb = trsm_stage_bytes(dtype, h->n, m);
  o->stage = sb ? (float *)take(sb) : nullptr;
  o->qmf = take(thin_q_bytes(m));
  return RHQR_OK;
}

__global__ void k_zero_mat(double *A, int64_t lda, int32_t rows, int32_t cols) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r < rows && c < cols) A[r + (int64_t)c * lda] = 0.0;
}

}  // namespace

// Sketch-space Householder QR of Z (L x m float64, copied to Zc, which is
// overwritten): S (Householder vectors, unit pivot), T, R.
int sketch_space_hqr(int32_t L, int32_t m, double *Zc, double *S, int64_t lds, double *T,
                     int64_t ldt, double *R, int64_t ldr, const LoopWs &w, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_mat, dim3((m + 255) / 256, m), dim3(256), 0, st, T, ldt, m, m);
  RHQR_HIP(hipGetLastError());
  LoopArgs a;
  a.kind = RHQR_SKETCH_IDENT;
  a.dtype = RHQR_F64;
  a.n = L;
  a.m = m;
  a.l = L - m;
  a.W = Zc;
  a.ldw = L;
  a.Z = Zc;  // Psi = I: the pre-sketch of column j+1 is column j+1 itself (unmodified at step j)
  a.ldz = L;
  a.S = S;
  a.lds = lds;
  a.T = T;
  a.ldt = ldt;
  a.R = R;
  a.ldr = ldr;
  a.scaling = RHQR_SCALE_UNIT_PIVOT;
  a.signs = nullptr;
  a.rows = nullptr;
  a.omega = nullptr;
  a.defer = 1;
  return run_column_loop(a, w, st);
}

extern "C" size_t recrhqr_workspace_size(rhqr_sketch_t h, int dtype, int32_t m) {
  if (!h || m != h->m || dtype < RHQR_F64 || dtype > RHQR_BF16) return 0;
  return rec_ws_bytes(h, dtype, m);
}

extern "C" int recrhqr_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, const void *d_W,
                              int64_t ldw, void *d_U, int64_t ldu, double *d_S, int64_t lds,
                              double *d_T, int64_t ldt, double *d_R, int64_t ldr, void *d_Q,
                              int64_t ldq, int mode, void *d_ws, size_t ws_bytes, void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (m != h->m) return -4;
  if (!d_W) return -5;
  if (ldw < n) return -6;
  if (mode == RHQR_REC_M && !d_U) return -7;
  if (d_U && ldu < n) return -8;
  const int32_t L = h->l + m;
  if (!d_S) return -9;
  if (lds < L) return -10;
  if (!d_T) return -11;
  if (ldt < m) return -12;
  if (!d_R) return -13;
  if (ldr < m) return -14;
  if (d_Q && ldq < n) return -16;
  if (mode != RHQR_REC_M && mode != RHQR_REC_RCHOL) return -17;
  if (mode == RHQR_REC_RCHOL && !d_Q) return -15;
  if (!d_ws) return -18;
  if (m > 1024) return RHQR_ERR_UNSUPPORTED;
  hipStream_t st = (hipStream_t)stream;
  RecWs w;
  int rc = rec_ws_carve(h, dtype, m, d_ws, ws_bytes, &w);
  if (rc) return rc;
  rc = launch_fill(w.loop.status, 16, st);
  if (rc) return rc;
  // single synchronisation: the sketch of every column
  rc = launch_sketch(h, dtype, n, m, d_W, ldw, w.Z, L, w.skws, w.skws_bytes, st);
  if (rc) return rc;
  RHQR_HIP(hipMemcpyAsync(w.Zc, w.Z, sizeof(double) * (size_t)L * m, hipMemcpyDeviceToDevice, st));
  rc = sketch_space_hqr(L, m, w.Zc, d_S, lds, d_T, ldt, d_R, ldr, w.loop, st);
  if (rc) return rc;
  if (mode == RHQR_REC_M) {
    const int64_t nent = (int64_t)m * m;
    hipLaunchKernelGGL(k_gram, dim3((nent + 15) / 16), dim3(1024), 0, st, m, L, d_S, lds, w.Z,
                       (int64_t)L, w.G);
    RHQR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_ttg, dim3((m + 255) / 256, m), dim3(256), 0, st, m, d_T, ldt, w.G, w.M);
    RHQR_HIP(hipGetLastError());
    const size_t es = dtype_size(dtype);
    rc = launch_trsm_blocked(dtype, (const char *)d_W + (size_t)m * es, ldw, n - m, m, w.M, m,
                             (char *)d_U + (size_t)m * es, ldu, w.coef, w.stage, st);
    if (rc) return rc;
    rc = launch_head_copy(dtype, d_U, ldu, m, d_S, lds, st);
    if (rc) return rc;
    if (d_Q)
      rc = launch_thin_q(dtype, n, m, d_U, ldu, d_S, lds, d_T, ldt, w.Mq, w.qmf, d_Q, ldq, st);
    return rc;
  }
  // randomized Cholesky QR: Q = W R^-1
  return launch_trsm_blocked(dtype, d_W, ldw, n, m, d_R, ldr, d_Q, ldq, w.coef, w.stage, st);
}
