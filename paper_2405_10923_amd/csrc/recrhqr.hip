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

// ------------------------------------------- sketch-space Householder QR
// Householder QR of the small L x m float64 sketch Z (overwritten),
// right-looking in panels of SQ_NB columns, two launches per panel.
// k_hqr_panel (one workgroup) factors the panel in LDS one column at a time
// (RHVector with Psi = I, Alg. 2: sigma, rho, gamma, alpha, beta; identity
// reflector when rho = 0), writes its vectors to S and extends T by the
// recursion of Prop. 3.2 (T_{:,j} = -beta_j T S^t s_j, in block form per
// panel).  k_hqr_trail (one workgroup per trailing column) applies the panel's
// block reflector, Z <- (I - S_p T_p^t S_p^t) Z.  Every reduction runs in a
// fixed order.  The same factorization as the column engine with Psi = I,
// in far fewer launches.
constexpr int SQ_NB = 8, SQ_TPB = 1024;
constexpr int SQ_MAXL = 2048;  // L + m at most: the panel (L x SQ_NB) and Y (m x SQ_NB) in LDS
constexpr int SQ_MAXM = 1024;  // largest m (recrhqr_factor rejects larger)
constexpr int SQ_RC = 8;       // rows per lane held in registers by a column pass (512 rows)

// sum over the workgroup of one value per thread, fixed order; all threads
// get the result
__device__ __forceinline__ double sq_block_sum(double v, double *red16) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  v = wave_sum(v);
  __syncthreads();  // red16 may still be read by the previous sum
  if (lane == 0) red16[w] = v;
  __syncthreads();
  double s = 0.0;
  for (int i = 0; i < SQ_TPB / 64; ++i) s += red16[i];
  return s;
}

__global__ void __launch_bounds__(SQ_TPB) k_hqr_panel(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, double *S, int64_t lds,
                                                      double *T, int64_t ldt, double *R,
                                                      int64_t ldr, int scaling, int32_t *status) {
  // panel: column c at Pn + c * rows, rows J .. L-1; after it, Y (J x SQ_NB)
  extern __shared__ double Pn[];
  __shared__ double red16[SQ_TPB / 64];
  __shared__ double redv[SQ_TPB / 64][SQ_NB];
  __shared__ double gv[SQ_MAXM];
  __shared__ double bet[SQ_NB];
  __shared__ double Tp[SQ_NB][SQ_NB];  // T_pp (upper triangle), also written to T
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = m - J < SQ_NB ? m - J : SQ_NB;
  const int rows = L - J;
  // the panel's rows J.. into LDS; its rows < J are final entries of R
  for (int e = tid; e < rows * nb; e += SQ_TPB) {
    const int r = e % rows, c = e / rows;
    Pn[c * rows + r] = Z[(J + r) + (int64_t)(J + c) * ldz];
  }
  for (int e = tid; e < J * nb; e += SQ_TPB) {
    const int r = e % J, c = e / J;
    R[r + (int64_t)(J + c) * ldr] = Z[r + (int64_t)(J + c) * ldz];
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const int j = J + c;
    double *x = Pn + c * rows;  // local row r is row J + r; the pivot is local row c
    double ss = 0.0;
    for (int r = c + tid; r < rows; r += SQ_TPB) ss += x[r] * x[r];
    ss = sq_block_sum(ss, red16);
    // RHVector scalars (every thread computes the same values)
    const double rho = sqrt(ss);
    const double yj = x[c];
    const double sigma = yj >= 0.0 ? 1.0 : -1.0;
    const bool ident = !(rho > 0.0);
    double gamma = 0.0, alpha = 1.0, beta = 0.0;
    if (!ident) {
      gamma = yj + sigma * rho;
      if (scaling == RHQR_SCALE_UNIT_PIVOT) {
        alpha = gamma;
        beta = fabs(gamma) / rho;
      } else {
        alpha = sqrt(rho * fabs(gamma));
        beta = 1.0;
      }
    }
    const double sr = sigma * rho;
    __syncthreads();  // every thread has read x[c]
    // R column j: rows J..j-1 from the panel, -sigma rho on the diagonal, zeros below
    for (int r = tid; r < m; r += SQ_TPB) {
      if (r >= J && r < j) R[r + (int64_t)j * ldr] = x[r - J];
      else if (r == j) R[r + (int64_t)j * ldr] = -sr;
      else if (r > j) R[r + (int64_t)j * ldr] = 0.0;
    }
    __syncthreads();  // the R entries above the pivot have been read
    // s_j in place of the column
    for (int r = tid; r < rows; r += SQ_TPB) {
      double sv = 0.0;
      if (r == c)
        sv = ident ? 1.0 : (scaling == RHQR_SCALE_UNIT_PIVOT ? 1.0 : gamma / alpha);
      else if (r > c)
        sv = ident ? 0.0 : x[r] / alpha;
      x[r] = sv;
    }
    if (tid == 0) {
      bet[c] = beta;
      Tp[c][c] = beta;
      T[j + (int64_t)j * ldt] = beta;
      if (ident) atomicCAS(status, 0, j + 1);
      if (!(isfinite(ss) && isfinite(yj))) atomicCAS(status + 1, 0, j + 1);
    }
    __syncthreads();
    // H_j = I - beta s_j s_j^t on the panel's later columns (rows >= j)
    const int nrem = nb - 1 - c;
    if (nrem > 0 && !ident) {
      double d[SQ_NB];
#pragma unroll
      for (int q = 0; q < SQ_NB; ++q) d[q] = 0.0;
      for (int r = c + tid; r < rows; r += SQ_TPB) {
        const double sv = x[r];
#pragma unroll
        for (int q = 0; q < SQ_NB; ++q)
          if (q < nrem) d[q] += sv * Pn[(c + 1 + q) * rows + r];
      }
#pragma unroll
      for (int q = 0; q < SQ_NB; ++q) {
        const double v = wave_sum(d[q]);
        if (lane == 0 && q < nrem) redv[w][q] = v;
      }
      __syncthreads();
      if (tid < nrem) {
        double sum = 0.0;
        for (int i = 0; i < SQ_TPB / 64; ++i) sum += redv[i][tid];
        gv[tid] = beta * sum;
      }
      __syncthreads();
      for (int e = tid; e < nrem * (rows - c); e += SQ_TPB) {
        const int q = e / (rows - c), r = c + e % (rows - c);
        Pn[(c + 1 + q) * rows + r] -= gv[q] * x[r];
      }
      __syncthreads();
    }
  }
  // the panel's vectors into S (zeros above the panel rows)
  for (int e = tid; e < L * nb; e += SQ_TPB) {
    const int r = e % L, c = e / L;
    S[r + (int64_t)(J + c) * lds] = r < J ? 0.0 : Pn[c * rows + (r - J)];
  }
  __syncthreads();
  // T columns J..J+nb-1, block form of the Prop. 3.2 recursion: the
  // panel's own block T_pp (g = S_p^t s_j over the panel, from LDS), then
  // T_{<J, p} = -T_{<J,<J} (S_{<J}^t S_p) T_pp.
  for (int c = 0; c < nb; ++c) {
    const double *xj = Pn + c * rows;
    // g_q = s_q^t s_j for the panel's q < c (rows >= J + c), one wave per q
    for (int q = w; q < c; q += SQ_TPB / 64) {
      const double *xq = Pn + q * rows;
      double v = 0.0;
      for (int r = c + lane; r < rows; r += 64) v += xq[r] * xj[r];
      v = wave_sum(v);
      if (lane == 0) gv[q] = v;
    }
    __syncthreads();
    if (tid < c) {
      double t = 0.0;
      for (int q = tid; q < c; ++q) t += Tp[tid][q] * gv[q];
      const double v = -bet[c] * t;
      Tp[tid][c] = v;
      T[(J + tid) + (int64_t)(J + c) * ldt] = v;
    }
    __syncthreads();
  }
  if (J > 0) {
    // X = S_{<J}^t S_p (rows >= J), one wave per earlier column p, into
    // T[p, J + c] as scratch
    for (int p = w; p < J; p += SQ_TPB / 64) {
      const double *sp = S + (int64_t)p * lds + J;
      double d[SQ_NB];
#pragma unroll
      for (int q = 0; q < SQ_NB; ++q) d[q] = 0.0;
      // the column's first SQ_RC * 64 rows are loaded at once, the rest
      // streamed; the sums run over rows in increasing order either way
      double sr[SQ_RC];
#pragma unroll
      for (int i = 0; i < SQ_RC; ++i) {
        const int r = lane + 64 * i;
        sr[i] = r < rows ? sp[r] : 0.0;
      }
#pragma unroll
      for (int i = 0; i < SQ_RC; ++i) {
        const int r = lane + 64 * i;
        if (r < rows) {
#pragma unroll
          for (int q = 0; q < SQ_NB; ++q)
            if (q < nb) d[q] += sr[i] * Pn[q * rows + r];
        }
      }
#pragma unroll 4
      for (int r = lane + 64 * SQ_RC; r < rows; r += 64) {
        const double sv = sp[r];
#pragma unroll
        for (int q = 0; q < SQ_NB; ++q)
          if (q < nb) d[q] += sv * Pn[q * rows + r];
      }
#pragma unroll
      for (int q = 0; q < SQ_NB; ++q) {
        const double v = wave_sum(d[q]);
        if (lane == 0 && q < nb) T[p + (int64_t)(J + q) * ldt] = v;
      }
    }
    __syncthreads();
    // Y = T_{<J,<J} X into LDS (after the panel), one wave per row p,
    // lanes over q >= p
    double *Yl = Pn + (size_t)SQ_NB * rows;
    for (int p = w; p < J; p += SQ_TPB / 64) {
      double t[SQ_NB];
#pragma unroll
      for (int c = 0; c < SQ_NB; ++c) t[c] = 0.0;
      for (int q = p + lane; q < J; q += 64) {
        const double tpq = T[p + (int64_t)q * ldt];
#pragma unroll
        for (int c = 0; c < SQ_NB; ++c)
          if (c < nb) t[c] += tpq * T[q + (int64_t)(J + c) * ldt];
      }
#pragma unroll
      for (int c = 0; c < SQ_NB; ++c) {
        const double v = wave_sum(t[c]);
        if (lane == 0) Yl[p * SQ_NB + c] = v;
      }
    }
    __syncthreads();
    // T_{<J, p} = -Y T_pp, row by row
    for (int p = tid; p < J; p += SQ_TPB) {
      double o[SQ_NB];
#pragma unroll
      for (int c = 0; c < SQ_NB; ++c) {
        double t = 0.0;
#pragma unroll
        for (int q = 0; q < SQ_NB; ++q)
          if (q <= c && c < nb) t += Yl[p * SQ_NB + q] * Tp[q][c];
        o[c] = -t;
      }
#pragma unroll
      for (int c = 0; c < SQ_NB; ++c)
        if (c < nb) T[p + (int64_t)(J + c) * ldt] = o[c];
    }
    __syncthreads();
  }
}

// trailing column k = J + nb + blockIdx.x of panel J: w = S_p^t Z_k,
// u = T_p^t w, Z_k -= S_p u (rows >= J), with the panel's vectors read from
// S.  One workgroup per column: every thread loads its rows (at most
// SQ_MAXL / TR_TPB) at once, the dot products are summed per wave and then
// over the waves in a fixed order.
constexpr int TR_TPB = 256;
constexpr int TR_RC = SQ_MAXL / TR_TPB;  // rows per thread
__global__ void __launch_bounds__(TR_TPB) k_hqr_trail(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, const double *S, int64_t lds,
                                                      const double *T, int64_t ldt) {
  __shared__ double red[TR_TPB / 64][SQ_NB];
  const int nb = m - J < SQ_NB ? m - J : SQ_NB;
  const int rows = L - J, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = J + nb + (int)blockIdx.x;
  if (k >= m) return;  // the whole workgroup
  const double *Sp = S + J + (int64_t)J * lds;  // Sp[r + q * lds]: panel vector q, row J + r
  double *zk = Z + (int64_t)k * ldz + J;
  double zr[TR_RC], d[SQ_NB];
#pragma unroll
  for (int q = 0; q < SQ_NB; ++q) d[q] = 0.0;
#pragma unroll
  for (int i = 0; i < TR_RC; ++i) {
    const int r = tid + TR_TPB * i;
    zr[i] = r < rows ? zk[r] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < TR_RC; ++i) {
    const int r = tid + TR_TPB * i;
    if (r < rows) {
#pragma unroll
      for (int q = 0; q < SQ_NB; ++q)
        if (q < nb) d[q] += Sp[r + (int64_t)q * lds] * zr[i];
    }
  }
#pragma unroll
  for (int q = 0; q < SQ_NB; ++q) {
    const double v = wave_sum(d[q]);
    if (lane == 0) red[w][q] = v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < SQ_NB; ++q) {
    static_assert(TR_TPB / 64 == 4, "four partial sums per value");
    d[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
  double u[SQ_NB];
#pragma unroll
  for (int c = 0; c < SQ_NB; ++c) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < SQ_NB; ++q)
      if (q <= c && c < nb) t += T[(J + q) + (int64_t)(J + c) * ldt] * d[q];
    u[c] = t;
  }
#pragma unroll
  for (int i = 0; i < TR_RC; ++i) {
    const int r = tid + TR_TPB * i;
    if (r < rows) {
      double zv = zr[i];
#pragma unroll
      for (int c = 0; c < SQ_NB; ++c)
        if (c < nb) zv -= Sp[r + (int64_t)c * lds] * u[c];
      zk[r] = zv;
    }
  }
}

}  // namespace

// Sketch-space Householder QR of Z (L x m float64, copied to Zc, which is
// overwritten): S (Householder vectors, unit pivot), T, R.
int sketch_space_hqr(int32_t L, int32_t m, double *Zc, double *S, int64_t lds, double *T,
                     int64_t ldt, double *R, int64_t ldr, const LoopWs &w, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_mat, dim3((m + 255) / 256, m), dim3(256), 0, st, T, ldt, m, m);
  RHQR_HIP(hipGetLastError());
  if (L + m <= SQ_MAXL) {  // the panel in LDS; two launches per panel
    const size_t lds_bytes = sizeof(double) * (size_t)(L + m) * SQ_NB;
    static bool attr_set = false;
    if (!attr_set) {
      RHQR_HIP(hipFuncSetAttribute((const void *)k_hqr_panel,
                                   hipFuncAttributeMaxDynamicSharedMemorySize,
                                   (int)(sizeof(double) * SQ_MAXL * SQ_NB)));
      attr_set = true;
    }
    for (int32_t J = 0; J < m; J += SQ_NB) {
      const int32_t nb = m - J < SQ_NB ? m - J : SQ_NB;
      RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_panel, dim3(1), dim3(SQ_TPB), lds_bytes, st, L, m, J, Zc,
                  (int64_t)L, S, lds, T, ldt, R, ldr, (int)RHQR_SCALE_UNIT_PIVOT, w.status);
      if (J + nb < m) {
        RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_trail, dim3((unsigned)(m - J - nb)), dim3(TR_TPB), 0, st,
                    L, m, J, Zc, (int64_t)L, (const double *)S, lds, (const double *)T, ldt);
      }
    }
    return RHQR_OK;
  }
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
  if (!h || m < 1 || m != h->m || dtype < RHQR_F64 || dtype > RHQR_BF16) return 0;
  return rec_ws_bytes(h, dtype, m);
}

extern "C" int recrhqr_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, const void *d_W,
                              int64_t ldw, void *d_U, int64_t ldu, double *d_S, int64_t lds,
                              double *d_T, int64_t ldt, double *d_R, int64_t ldr, void *d_Q,
                              int64_t ldq, int mode, void *d_ws, size_t ws_bytes, void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (m < 1 || m != h->m) return -4;
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
