// recRHQR (Alg. 6): RHQR reconstructed from the Householder QR of the sketch.
//
//   Z = Psi W                                  (one multi-column sketch pass)
//   S, T, R = HouseholderQR(Z)                 (float64, on the device: the
//                                               column engine run with Psi = I)
//   M = ut(T^t S^t Z)   (= -T U_1^t R, Sec. 3.3)
//   U_2 M = W_2         (forward substitution, launch_trsm_blocked)
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
// right-looking in panels of NB columns (16, or 8 for tall sketches).
// k_hqr_panel (one workgroup) factors the panel in LDS one column at a time
// (RHVector with Psi = I, Alg. 2: sigma, rho, gamma, alpha, beta; identity
// reflector when rho = 0), writes its vectors to S and the panel's diagonal
// block of T (Prop. 3.2 recursion within the panel).  Thread t owns the panel
// rows r = t mod HQ_TPB for every column, so a column costs two workgroup
// reductions (its norm, then its products with the later panel columns) and
// no other synchronisation.  k_hqr_trail (one workgroup per trailing column)
// applies the panel's block reflector, Z <- (I - S_p T_pp^t S_p^t) Z.  After
// the last panel the off-diagonal blocks of T follow from the Gram matrix
// G = S^t S: T_{<J, p} = -T_{<J,<J} G_{<J, p} T_pp (Prop. 3.2 in block form),
// one launch per panel.  Every reduction runs in a fixed order.  The same
// factorization as the column engine with Psi = I, in far fewer launches.
constexpr int HQ_TPB = 256;
constexpr int HQ_W = HQ_TPB / 64;
constexpr int SQ_MAXL = 2048;  // L + m at most on this path (else the column engine)
constexpr int SQ_MAXM = 1024;  // largest m (recrhqr_factor rejects larger)
constexpr size_t HQ_LDS_MAX = 150 * 1024;  // dynamic LDS budget of the panel kernel

// panel width for an L-row sketch: 16 when the panel fits the LDS budget
inline int hqr_nb(int32_t L, int32_t m) {
  return (size_t)L * 16 * sizeof(double) <= HQ_LDS_MAX && m <= 512 ? 16 : 8;
}

template <int NB>
__global__ void __launch_bounds__(HQ_TPB) k_hqr_panel(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, double *S, int64_t lds,
                                                      double *T, int64_t ldt, double *R,
                                                      int64_t ldr, int scaling, int32_t *status) {
  // panel: column c at Pn + c * rows, local row r is row J + r
  extern __shared__ double Pn[];
  __shared__ double nrm[2][HQ_W];
  __shared__ double red[2][HQ_W][NB];
  __shared__ double gp[NB][NB];  // s_q^t s_c over the panel (q < c)
  __shared__ double bet[NB], spv[NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = m - J < NB ? m - J : NB;
  const int rows = L - J;
  for (int e = tid; e < rows * nb; e += HQ_TPB) {
    const int r = e % rows, c = e / rows;
    Pn[c * rows + r] = Z[(J + r) + (int64_t)(J + c) * ldz];
  }
  for (int e = tid; e < J * nb; e += HQ_TPB) {
    const int r = e % J, c = e / J;
    R[r + (int64_t)(J + c) * ldr] = Z[r + (int64_t)(J + c) * ldz];
  }
  __syncthreads();
  for (int c = 0; c < nb; ++c) {
    const int j = J + c, b = c & 1;
    double *x = Pn + c * rows;  // the pivot is local row c
    double ss = 0.0;
    for (int r = tid; r < rows; r += HQ_TPB) ss += r >= c ? x[r] * x[r] : 0.0;
    ss = wave_sum(ss);
    if (lane == 0) nrm[b][w] = ss;
    __syncthreads();  // the norm partials; the pivot (updated by its owner) is final
    ss = 0.0;
#pragma unroll
    for (int i = 0; i < HQ_W; ++i) ss += nrm[b][i];
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
    // R column j (rows J..m-1): the final entries above the pivot, -sigma rho
    // on the diagonal, zeros below; local row r is owned by thread r mod HQ_TPB
    for (int r = tid; r < m - J; r += HQ_TPB)
      R[(J + r) + (int64_t)j * ldr] = r < c ? x[r] : (r == c ? -sr : 0.0);
    // s_j in place of the column (own rows > c); the pivot entry is written
    // after the column loop, since every thread reads the pivot above
    const double spiv = ident ? 1.0 : (scaling == RHQR_SCALE_UNIT_PIVOT ? 1.0 : gamma / alpha);
    for (int r = tid; r < rows; r += HQ_TPB)
      if (r > c) x[r] = ident ? 0.0 : x[r] / alpha;
    if (tid == 0) {
      spv[c] = spiv;
      bet[c] = beta;
      if (ident) atomicCAS(status, 0, j + 1);
      if (!(isfinite(ss) && isfinite(yj))) atomicCAS(status + 1, 0, j + 1);
    }
    // H_j = I - beta s_j s_j^t on the panel's later columns (own rows >= c)
    const int nrem = nb - 1 - c;
    if (nrem > 0) {  // uniform
      double d[NB];
#pragma unroll
      for (int q = 0; q < NB; ++q) d[q] = 0.0;
      for (int r = tid; r < rows; r += HQ_TPB) {
        if (r < c) continue;
        const double sv = r == c ? spiv : x[r];
#pragma unroll
        for (int q = 0; q < NB - 1; ++q)
          if (q < nrem) d[q] += sv * Pn[(c + 1 + q) * rows + r];
      }
#pragma unroll
      for (int q = 0; q < NB - 1; ++q) {
        if (q < nrem) {
          const double v = wave_sum(d[q]);
          if (lane == 0) red[b][w][q] = v;
        }
      }
      __syncthreads();  // the product partials
      double gq[NB];
#pragma unroll
      for (int q = 0; q < NB - 1; ++q) {
        double s = 0.0;
#pragma unroll
        for (int i = 0; i < HQ_W; ++i) s += q < nrem ? red[b][i][q] : 0.0;
        gq[q] = beta * s;
      }
      for (int r = tid; r < rows; r += HQ_TPB) {
        if (r < c) continue;
        const double sv = r == c ? spiv : x[r];
#pragma unroll
        for (int q = 0; q < NB - 1; ++q)
          if (q < nrem) Pn[(c + 1 + q) * rows + r] -= gq[q] * sv;
      }
    }
  }
  __syncthreads();
  if (tid < nb) Pn[tid * rows + tid] = spv[tid];
  __syncthreads();
  // the panel's vectors into S (zeros above each pivot: the panel column
  // still holds its R entries there)
  for (int e = tid; e < L * nb; e += HQ_TPB) {
    const int r = e % L, c = e / L;
    S[r + (int64_t)(J + c) * lds] = r < J + c ? 0.0 : Pn[c * rows + (r - J)];
  }
  // T_pp: g_{q,c} = s_q^t s_c over rows >= c (s_c is zero above its pivot),
  // one wave per pair
  for (int pr = w; pr < nb * nb; pr += HQ_W) {
    const int q = pr % nb, c = pr / nb;
    if (q >= c) continue;  // uniform across the wave
    const double *xq = Pn + q * rows, *xc = Pn + c * rows;
    double v = 0.0;
    for (int r = c + lane; r < rows; r += 64) v += xq[r] * xc[r];
    v = wave_sum(v);
    if (lane == 0) gp[q][c] = v;
  }
  __syncthreads();
  // row q of T_pp on lane q: T_qq = beta_q, T_qc = -beta_c sum_{q <= k < c} T_qk g_kc
  if (w == 0 && lane < nb) {
    const int q = lane;
    double tq[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      double v = 0.0;
      if (c < nb) {
        if (c == q) {
          v = bet[c];
        } else if (c > q) {
          double t = 0.0;
#pragma unroll
          for (int k = 0; k < NB; ++k)
            if (k < c && k >= q) t += tq[k] * gp[k][c];
          v = -bet[c] * t;
        }
        if (c >= q) T[(J + q) + (int64_t)(J + c) * ldt] = v;
      }
      tq[c] = v;
    }
  }
}

// trailing column k = J + nb + blockIdx.x of panel J: w = S_p^t Z_k,
// u = T_pp^t w, Z_k -= S_p u (rows >= J), with the panel's vectors read from
// S.  One workgroup per column: every thread loads its rows (at most
// SQ_MAXL / TR_TPB) at once, the dot products are summed per wave and then
// over the waves in a fixed order.
constexpr int TR_TPB = 256;
constexpr int TR_RC = SQ_MAXL / TR_TPB;  // rows per thread
template <int NB>
__global__ void __launch_bounds__(TR_TPB) k_hqr_trail(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, const double *S, int64_t lds,
                                                      const double *T, int64_t ldt) {
  __shared__ double red[TR_TPB / 64][NB];
  const int nb = m - J < NB ? m - J : NB;
  const int rows = L - J, tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int k = J + nb + (int)blockIdx.x;
  if (k >= m) return;  // the whole workgroup
  const double *Sp = S + J + (int64_t)J * lds;  // Sp[r + q * lds]: panel vector q, row J + r
  double *zk = Z + (int64_t)k * ldz + J;
  double zr[TR_RC], d[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) d[q] = 0.0;
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
      for (int q = 0; q < NB; ++q)
        if (q < nb) d[q] += Sp[r + (int64_t)q * lds] * zr[i];
    }
  }
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    const double v = wave_sum(d[q]);
    if (lane == 0) red[w][q] = v;
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NB; ++q) {
    static_assert(TR_TPB / 64 == 4, "four partial sums per value");
    d[q] = (red[0][q] + red[1][q]) + (red[2][q] + red[3][q]);
  }
  double u[NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    double t = 0.0;
#pragma unroll
    for (int q = 0; q < NB; ++q)
      if (q <= c && c < nb) t += T[(J + q) + (int64_t)(J + c) * ldt] * d[q];
    u[c] = t;
  }
#pragma unroll
  for (int i = 0; i < TR_RC; ++i) {
    const int r = tid + TR_TPB * i;
    if (r < rows) {
      double zv = zr[i];
#pragma unroll
      for (int c = 0; c < NB; ++c)
        if (c < nb) zv -= Sp[r + (int64_t)c * lds] * u[c];
      zk[r] = zv;
    }
  }
}

// T_{<J, p} = -(T_{<J,<J} G_{<J, p}) T_pp for the panel p = J..J+nb-1, with
// G = S^t S (ld m).  One workgroup: Y = T_{<J,<J} G_{<J,p} into LDS (one
// thread per entry, sum over q in increasing order), then the product with
// the panel's diagonal block.  T_{<J,<J} comes from the earlier launches.
constexpr int TF_TPB = 1024;
template <int NB>
__global__ void __launch_bounds__(TF_TPB) k_hqr_tfill(int32_t m, int32_t J,
                                                      const double *__restrict__ G,
                                                      double *__restrict__ T, int64_t ldt) {
  extern __shared__ double Y[];  // J x nb, ld J
  const int nb = m - J < NB ? m - J : NB;
  for (int e = threadIdx.x; e < J * nb; e += TF_TPB) {
    const int p = e % J, c = e / J;
    const double *g = G + (int64_t)(J + c) * m;
    double y = 0.0;
    for (int q = p; q < J; ++q) y += T[p + (int64_t)q * ldt] * g[q];
    Y[p + c * J] = y;
  }
  __syncthreads();
  for (int e = threadIdx.x; e < J * nb; e += TF_TPB) {
    const int p = e % J, c = e / J;
    double t = 0.0;
    for (int q = 0; q <= c; ++q) t += Y[p + q * J] * T[(J + q) + (int64_t)(J + c) * ldt];
    T[p + (int64_t)(J + c) * ldt] = -t;
  }
}

}  // namespace

// Sketch-space Householder QR of Z (L x m float64, copied to Zc, which is
// overwritten): S (Householder vectors, unit pivot), T, R.  G: m x m float64
// scratch (S^t S).
int sketch_space_hqr(int32_t L, int32_t m, double *Zc, double *S, int64_t lds, double *T,
                     int64_t ldt, double *R, int64_t ldr, double *G, const LoopWs &w,
                     hipStream_t st) {
  hipLaunchKernelGGL(k_zero_mat, dim3((m + 255) / 256, m), dim3(256), 0, st, T, ldt, m, m);
  RHQR_HIP(hipGetLastError());
  if (L + m <= SQ_MAXL) {  // the panel in LDS; two launches per panel
    const int NBv = hqr_nb(L, m);
    static bool attr_set = false;
    if (!attr_set) {
      RHQR_HIP(hipFuncSetAttribute((const void *)k_hqr_panel<16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)HQ_LDS_MAX));
      RHQR_HIP(hipFuncSetAttribute((const void *)k_hqr_panel<8>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)HQ_LDS_MAX));
      RHQR_HIP(hipFuncSetAttribute((const void *)k_hqr_tfill<16>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)HQ_LDS_MAX));
      RHQR_HIP(hipFuncSetAttribute((const void *)k_hqr_tfill<8>,
                                   hipFuncAttributeMaxDynamicSharedMemorySize, (int)HQ_LDS_MAX));
      attr_set = true;
    }
    const size_t lds_bytes = sizeof(double) * (size_t)L * NBv;
    for (int32_t J = 0; J < m; J += NBv) {
      const int32_t nb = m - J < NBv ? m - J : NBv;
      if (NBv == 16)
        RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_panel<16>, dim3(1), dim3(HQ_TPB), lds_bytes, st, L, m, J,
                    Zc, (int64_t)L, S, lds, T, ldt, R, ldr, (int)RHQR_SCALE_UNIT_PIVOT, w.status);
      else
        RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_panel<8>, dim3(1), dim3(HQ_TPB), lds_bytes, st, L, m, J,
                    Zc, (int64_t)L, S, lds, T, ldt, R, ldr, (int)RHQR_SCALE_UNIT_PIVOT, w.status);
      RHQR_HIP(hipGetLastError());
      if (J + nb < m) {
        const dim3 g((unsigned)(m - J - nb));
        if (NBv == 16)
          RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_trail<16>, g, dim3(TR_TPB), 0, st, L, m, J, Zc,
                      (int64_t)L, (const double *)S, lds, (const double *)T, ldt);
        else
          RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_trail<8>, g, dim3(TR_TPB), 0, st, L, m, J, Zc,
                      (int64_t)L, (const double *)S, lds, (const double *)T, ldt);
        RHQR_HIP(hipGetLastError());
      }
    }
    if (m > NBv) {
      const int64_t nent = (int64_t)m * m;
      RHQR_LAUNCH(RHQR_PROF_HQR, k_gram, dim3((nent + 15) / 16), dim3(1024), 0, st, m, L,
                  (const double *)S, lds, (const double *)S, lds, G);
      RHQR_HIP(hipGetLastError());
      for (int32_t J = NBv; J < m; J += NBv) {
        const int32_t nb = m - J < NBv ? m - J : NBv;
        const size_t yb = sizeof(double) * (size_t)J * nb;
        if (NBv == 16)
          RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_tfill<16>, dim3(1), dim3(TF_TPB), yb, st, m, J,
                      (const double *)G, T, ldt);
        else
          RHQR_LAUNCH(RHQR_PROF_HQR, k_hqr_tfill<8>, dim3(1), dim3(TF_TPB), yb, st, m, J,
                      (const double *)G, T, ldt);
        RHQR_HIP(hipGetLastError());
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
  rc = sketch_space_hqr(L, m, w.Zc, d_S, lds, d_T, ldt, d_R, ldr, w.G, w.loop, st);
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
