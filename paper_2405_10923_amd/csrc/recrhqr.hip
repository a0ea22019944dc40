// recRHQR (Alg. 6): RHQR reconstructed from the Householder QR of the sketch.
//
//   Z = Psi W                                  (one multi-column sketch pass)
//   S, T, R = HouseholderQR(Z)                 (float64, on the device: the
//                                               column engine run with Psi = I)
//   M = ut(T^t S^t Z)   (= -T U_1^t R, Sec. 3.3)
//   U_2 M = W_2         (row-wise forward substitution, tall kernel k_trsm)
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

// X M = B for X (rows r0..r1 of an n x m matrix), M upper triangular m x m.
// A workgroup owns TR rows; the TR x m tile lives in LDS (column-major, ld TR)
// and is solved in column blocks of 16:
//   block update  A_blk = B_blk - X_{:, <cb} M_{<cb, blk}   (256 threads, 2 x 1 each)
//   block solve   x_c = (a_c - sum_{cb <= p < c} x_p M_{p,c}) / M_{c,c}   (one thread per row)
// The M block column is staged in LDS.  Rows are independent: each row's
// result is the float64 (float32 for low precision) forward substitution.
constexpr int TR = 32, TNB = 16;

template <typename ST>
__global__ void __launch_bounds__(256) k_trsm(const ST *__restrict__ B, int64_t ldb, int64_t r0,
                                              int64_t r1, int32_t m, const double *__restrict__ M,
                                              int64_t ldm, ST *__restrict__ X, int64_t ldx) {
  using CT = typename CompT<ST>::type;
  extern __shared__ unsigned char smem_raw[];
  CT *tile = reinterpret_cast<CT *>(smem_raw);  // TR x m
  CT *Mb = tile + (size_t)TR * m;               // m x TNB (row k, column c -> Mb[k*TNB + c])
  const int64_t rb = r0 + (int64_t)blockIdx.x * TR;
  const int nr = (int)(r1 - rb < TR ? r1 - rb : TR);
  // load the row tile
  for (int e = threadIdx.x; e < TR * m; e += blockDim.x) {
    const int r = e % TR, cidx = e / TR;
    tile[e] = r < nr ? cvt_in<CT>(B[rb + r + (int64_t)cidx * ldb]) : (CT)0;
  }
  const int tc = threadIdx.x & (TNB - 1);
  const int tr = (threadIdx.x >> 4) * 2;
  for (int cb = 0; cb < m; cb += TNB) {
    const int nb = m - cb < TNB ? m - cb : TNB;
    __syncthreads();
    for (int e = threadIdx.x; e < (cb + nb) * TNB; e += blockDim.x) {
      const int k = e / TNB, cc = e % TNB;
      Mb[e] = cc < nb ? (CT)M[k + (int64_t)(cb + cc) * ldm] : (CT)0;
    }
    __syncthreads();
    if (tc < nb) {
      const int col = cb + tc;
      CT a0 = tile[tr + (size_t)col * TR], a1 = tile[tr + 1 + (size_t)col * TR];
      for (int k = 0; k < cb; ++k) {
        const CT mk = Mb[k * TNB + tc];
        a0 -= tile[tr + (size_t)k * TR] * mk;
        a1 -= tile[tr + 1 + (size_t)k * TR] * mk;
      }
      tile[tr + (size_t)col * TR] = a0;
      tile[tr + 1 + (size_t)col * TR] = a1;
    }
    __syncthreads();
    if (threadIdx.x < TR) {
      const int r = threadIdx.x;
      for (int c = 0; c < nb; ++c) {
        CT a = tile[r + (size_t)(cb + c) * TR];
        for (int p = 0; p < c; ++p) a -= tile[r + (size_t)(cb + p) * TR] * Mb[(cb + p) * TNB + c];
        tile[r + (size_t)(cb + c) * TR] = a / Mb[(cb + c) * TNB + c];
      }
    }
  }
  __syncthreads();
  for (int e = threadIdx.x; e < TR * m; e += blockDim.x) {
    const int r = e % TR, cidx = e / TR;
    if (r < nr) X[rb + r + (int64_t)cidx * ldx] = cvt_out<ST>((double)tile[e]);
  }
}

template <typename ST>
__global__ void k_head_copy(ST *U, int64_t ldu, int32_t m, const double *S, int64_t lds) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k < m) U[k + (int64_t)c * ldu] = cvt_out<ST>(S[k + (int64_t)c * lds]);
}

template <typename ST>
int trsm_typed(const void *B, int64_t ldb, int64_t r0, int64_t r1, int32_t m, const double *M,
               int64_t ldm, void *X, int64_t ldx, hipStream_t st) {
  using CT = typename CompT<ST>::type;
  if (r1 <= r0) return RHQR_OK;
  const size_t shm = ((size_t)TR * m + (size_t)m * TNB) * sizeof(CT);
  if (shm > 160 * 1024) return RHQR_ERR_UNSUPPORTED;
  RHQR_HIP(hipFuncSetAttribute((const void *)k_trsm<ST>, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm));
  const int64_t g = (r1 - r0 + TR - 1) / TR;
  hipLaunchKernelGGL((k_trsm<ST>), dim3(g), dim3(256), shm, st, (const ST *)B, ldb, r0, r1, m, M,
                     ldm, (ST *)X, ldx);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

int launch_trsm(int dtype, const void *B, int64_t ldb, int64_t r0, int64_t r1, int32_t m,
                const double *M, int64_t ldm, void *X, int64_t ldx, hipStream_t st) {
  switch (dtype) {
    case RHQR_F64: return trsm_typed<double>(B, ldb, r0, r1, m, M, ldm, X, ldx, st);
    case RHQR_F32: return trsm_typed<float>(B, ldb, r0, r1, m, M, ldm, X, ldx, st);
    case RHQR_F16: return trsm_typed<__half>(B, ldb, r0, r1, m, M, ldm, X, ldx, st);
    case RHQR_BF16: return trsm_typed<__hip_bfloat16>(B, ldb, r0, r1, m, M, ldm, X, ldx, st);
  }
  return RHQR_ERR_UNSUPPORTED;
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
  double *Z, *Zc, *G, *M, *Mq;
  void *skws;
  size_t skws_bytes;
};

size_t rec_ws_bytes(const rhqr_sketch_s *h, int32_t m) {
  const int32_t L = h->l + m;
  size_t b = align_up(loop_ws_bytes(RHQR_SKETCH_IDENT, RHQR_F64, L, m, h->l));
  b += 2 * align_up(sizeof(double) * (size_t)L * m);
  b += 3 * align_up(sizeof(double) * (size_t)m * m);
  b += align_up(sketch_ws_bytes(h, m));
  return b;
}

int rec_ws_carve(const rhqr_sketch_s *h, int32_t m, void *ws, size_t bytes, RecWs *o) {
  if (bytes < rec_ws_bytes(h, m)) return RHQR_ERR_WORKSPACE;
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
  return rec_ws_bytes(h, m);
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
  int rc = rec_ws_carve(h, m, d_ws, ws_bytes, &w);
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
    rc = launch_trsm(dtype, (const char *)d_W + (size_t)m * es, ldw, 0, n - m, m, w.M, m,
                     (char *)d_U + (size_t)m * es, ldu, st);
    if (rc) return rc;
    rc = launch_head_copy(dtype, d_U, ldu, m, d_S, lds, st);
    if (rc) return rc;
    if (d_Q) rc = launch_thin_q(dtype, n, m, d_U, ldu, d_S, lds, d_T, ldt, w.Mq, d_Q, ldq, st);
    return rc;
  }
  // randomized Cholesky QR: Q = W R^-1
  return launch_trsm(dtype, d_W, ldw, 0, n, m, d_R, ldr, d_Q, ldq, st);
}
