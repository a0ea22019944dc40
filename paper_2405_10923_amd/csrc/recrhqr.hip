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
#include <type_traits>

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
// right-looking in panels of NB = 8 columns, two launches per panel.  (The
// column steps are unrolled per panel column: panels of 16 make four times the
// straight-line code per launch and measured 3 % slower per call at
// 2^20 x 128, l = 512, for half the launches.)
// k_hqr_panel (one workgroup of HQ_TPB threads) factors the panel one column
// at a time (RHVector with Psi = I, Alg. 2: sigma, rho, gamma, alpha, beta;
// identity reflector when rho = 0) with the panel in registers: thread t holds
// rows t + HQ_TPB i of every panel column, so a column costs two workgroup
// reductions (its norm; its products with the later panel columns, summed
// eight at a time per wave) and nothing else.  Then it writes the panel's
// vectors to S, its columns of R and the diagonal block T_pp (Prop. 3.2
// recursion within the panel).
// k_hqr_trail runs three kinds of workgroups: one per trailing column, which
// applies the panel's block reflector, Z <- (I - S_p T_pp^t S_p^t) Z; one per
// four earlier columns q, the products X_p = S_{<J}^t S_p (one wave per q);
// and one per sixteen rows of the previous panel's off-diagonal block of T,
// T_{<J', p'} = -(T_{<J',<J'} X_p') T_p'p' (Prop. 3.2 in block form), which is
// needed only at the end.  Every reduction runs in a fixed order.  The same
// factorization as the column engine with Psi = I, in far fewer launches.
constexpr int HQ_TPB = 256;
constexpr int HQ_W = HQ_TPB / 64;
constexpr int SQ_MAXL = 2048;  // L + m at most on this path (else the column engine)
constexpr int SQ_MAXM = 1024;  // largest m (recrhqr_factor rejects larger)


// f(integral_constant<int, I>) for I = B .. E-1, in order
template <int B, int E, typename F> __device__ __forceinline__ void static_for(F &&f) {
  if constexpr (B < E) {
    f(std::integral_constant<int, B>{});
    static_for<B + 1, E>(f);
  }
}

template <int NB, int RPT>
__global__ void __launch_bounds__(HQ_TPB) k_hqr_panel(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, double *S, int64_t lds,
                                                      double *T, int64_t ldt, double *R,
                                                      int64_t ldr, int scaling, int32_t *status) {
  __shared__ double nrm[2][HQ_W], pv[2];
  __shared__ double red[2][HQ_W][NB];
  __shared__ double gp[NB][NB];  // s_q^t s_c over the panel (q < c)
  __shared__ double bet[NB], dg[NB];
  __shared__ int flags[NB];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int nb = m - J < NB ? m - J : NB;
  const int rows = L - J;
  // own rows r_i = tid + HQ_TPB i of every column, loaded together (clamped
  // indices; rows beyond the sketch and columns beyond nb hold zeros)
  double P[RPT][NB];
#pragma unroll
  for (int c = 0; c < NB; ++c) {
    const double *zc = Z + (int64_t)(J + (c < nb ? c : nb - 1)) * ldz + J;
#pragma unroll
    for (int i = 0; i < RPT; ++i) {
      const int r = tid + HQ_TPB * i;
      const double v = zc[r < rows ? r : rows - 1];
      P[i][c] = (r < rows && c < nb) ? v : 0.0;
    }
  }
  // the final entries of R above the panel
  for (int r = tid; r < J; r += HQ_TPB) {
    double v[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) v[c] = Z[r + (int64_t)(J + (c < nb ? c : nb - 1)) * ldz];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) R[r + (int64_t)(J + c) * ldr] = v[c];
  }
  // one column step per compile-time c (the panel stays in registers)
  static_for<0, NB>([&](auto cc) {
    constexpr int c = decltype(cc)::value;
    if (c < nb) {  // uniform
      const int b = c & 1;
      // the norm of rows >= c; the pivot (row c, thread c) to LDS
      double ss = 0.0;
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + HQ_TPB * i;
        if (r >= c && r < rows) ss += P[i][c] * P[i][c];
      }
      ss = wave_sum(ss);
      if (lane == 0) nrm[b][w] = ss;
      if (tid == c) pv[b] = P[0][c];
      __syncthreads();
      ss = 0.0;
#pragma unroll
      for (int k = 0; k < HQ_W; ++k) ss += nrm[b][k];
      // RHVector scalars (every thread computes the same values)
      const double rho = sqrt(ss);
      const double yj = pv[b];
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
      // s_j in place of rows >= c (the rows above keep their R entries),
      // scaled by one reciprocal of alpha
      const double ia = 1.0 / alpha;
      const double spiv = ident ? 1.0 : (scaling == RHQR_SCALE_UNIT_PIVOT ? 1.0 : gamma * ia);
#pragma unroll
      for (int i = 0; i < RPT; ++i) {
        const int r = tid + HQ_TPB * i;
        if (r == c) P[i][c] = spiv;
        else if (r > c && r < rows) P[i][c] = ident ? 0.0 : P[i][c] * ia;
      }
      if (tid == 0) {
        bet[c] = beta;
        dg[c] = -sigma * rho;
        flags[c] = (ident ? 1 : 0) | (!(isfinite(ss) && isfinite(yj)) ? 2 : 0);
      }
      // H_j = I - beta s_j s_j^t on the panel's later columns (rows >= c),
      // and g_{q,c} = s_q^t s_c for the earlier ones (final since their own
      // steps; s_c is zero above its pivot), which T_pp needs: the products
      // with every panel column over rows >= c, reduced together
      if (c > 0 || c + 1 < nb) {  // uniform
        double d[NB];
#pragma unroll
        for (int q = 0; q < NB; ++q) d[q] = 0.0;
#pragma unroll
        for (int i = 0; i < RPT; ++i) {
          const int r = tid + HQ_TPB * i;
          if (r >= c && r < rows) {
#pragma unroll
            for (int q = 0; q < NB; ++q)
              if (q != c) d[q] += P[i][c] * P[i][q];
          }
        }
        // wave sums eight columns at a time: lane L holds the sum of column
        // 8 h + (L >> 3) of group h
#pragma unroll
        for (int h = 0; h < NB / 8; ++h) {
          double v8[8];
#pragma unroll
          for (int k = 0; k < 8; ++k) v8[k] = d[8 * h + k];
          const double tot = wave_sum8(v8);
          if ((lane & 7) == 0) red[b][w][8 * h + (lane >> 3)] = tot;
        }
        __syncthreads();
        // lane q (mod NB) sums column q over the waves in order; every thread
        // then reads the sums from those lanes
        double sq = 0.0;
#pragma unroll
        for (int k = 0; k < HQ_W; ++k) sq += red[b][k][lane & (NB - 1)];
        if (w == 0 && lane < c) gp[lane][c] = sq;
#pragma unroll
        for (int q = c + 1; q < NB; ++q) {
          const double g = beta * lane_read(sq, q);
#pragma unroll
          for (int i = 0; i < RPT; ++i) {
            const int r = tid + HQ_TPB * i;
            if (r >= c && r < rows) P[i][q] -= g * P[i][c];
          }
        }
      }
    }
  });
  // R columns J..J+nb-1, rows J..m-1 (the entries above each pivot, -sigma
  // rho on the diagonal, zeros below) and S (the vectors: zeros above each
  // pivot and above the panel), straight from the registers
#pragma unroll
  for (int i = 0; i < RPT; ++i) {
    const int r = tid + HQ_TPB * i;
#pragma unroll
    for (int c = 0; c < NB; ++c) {
      if (c >= nb) continue;
      if (r < m - J) R[(J + r) + (int64_t)(J + c) * ldr] = r < c ? P[i][c] : (r == c ? dg[c] : 0.0);
      if (r < rows) S[(J + r) + (int64_t)(J + c) * lds] = r < c ? 0.0 : P[i][c];
    }
  }
  for (int r = tid; r < J; r += HQ_TPB) {
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) S[r + (int64_t)(J + c) * lds] = 0.0;
  }
  if (tid == 0) {  // in column order: the first breakdown is the one kept
    for (int c = 0; c < nb; ++c) {
      if (flags[c] & 1) atomicCAS(status, 0, J + c + 1);
      if (flags[c] & 2) atomicCAS(status + 1, 0, J + c + 1);
    }
  }
  __syncthreads();  // g_{q,c} of the last steps
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

// The trail launch of panel J (columns J..J+nb-1), workgroups in three
// ranges:
//  [0, ntrail): trailing column k = J + nb + b: w = S_p^t Z_k, u = T_pp^t w,
//    Z_k -= S_p u (rows >= J), with the panel's vectors read from S.  Every
//    thread loads its rows (at most SQ_MAXL / TR_TPB) at once, the dot
//    products are summed per wave and then over the waves in a fixed order.
//  [ntrail, ntrail + nx): X_p = S_{<J}^t S_p (J x nb, ld m) into Xc, one wave
//    per earlier column q (rows >= J; the panel's vectors are zero above J).
//  the rest: rows p0 .. p0 + TF_ROWS - 1 of the off-diagonal block of T of
//    panel Jt (columns Jt..Jt+nbt-1): T_{<Jt, p} = -(T_{<Jt,<Jt} X) T_pp with
//    X = Xt from that panel's trail launch; each row of Y = T_{<Jt,<Jt} X by
//    one wave (lanes over the inner index, eight columns per butterfly).
// RC: rows of the trailing columns per thread (the launch's L - J rows).
constexpr int TR_TPB = 256;
constexpr int TR_MAXRC = SQ_MAXL / TR_TPB;  // rows per thread at most
constexpr int TF_ROWS = 16;                 // rows of T per workgroup
template <int NB, int RC>
__global__ void __launch_bounds__(TR_TPB) k_hqr_trail(int32_t L, int32_t m, int32_t J, double *Z,
                                                      int64_t ldz, const double *S, int64_t lds,
                                                      double *T, int64_t ldt, int ntrail, int nx,
                                                      double *__restrict__ Xc, int32_t Jt,
                                                      const double *__restrict__ Xt) {
  __shared__ double red[TR_TPB / 64][NB];
  __shared__ double tpp[NB][NB];
  __shared__ double yv[TF_ROWS][NB + 1];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int bid = (int)blockIdx.x;
  if (bid >= ntrail + nx) {
    // ---- off-diagonal block of T of panel Jt: rows p0 .. p0 + TF_ROWS - 1 (< Jt)
    const int nbt = m - Jt < NB ? m - Jt : NB;
    const int p0 = (bid - ntrail - nx) * TF_ROWS;
    if (tid < NB * NB) {
      const int q = tid % NB, c = tid / NB;
      tpp[q][c] = (q < nbt && c < nbt && q <= c) ? T[(Jt + q) + (int64_t)(Jt + c) * ldt] : 0.0;
    }
    static_assert(TF_ROWS * NB <= TR_TPB, "one thread per entry of the block");
    static_assert(NB % 8 == 0, "eight columns per butterfly");
    for (int pr = w; pr < TF_ROWS; pr += TR_TPB / 64) {
      const int p = p0 + pr;
      double yc[NB];
#pragma unroll
      for (int c = 0; c < NB; ++c) yc[c] = 0.0;
      for (int q = p + lane; q < Jt; q += 64) {  // p >= Jt: no term (uniform per wave)
        const double t = T[p + (int64_t)q * ldt];
#pragma unroll
        for (int c = 0; c < NB; ++c)
          if (c < nbt) yc[c] += t * Xt[q + (int64_t)c * m];
      }
#pragma unroll
      for (int h = 0; h < NB / 8; ++h) {
        double v8[8];
#pragma unroll
        for (int k = 0; k < 8; ++k) v8[k] = yc[8 * h + k];
        const double tot = wave_sum8(v8);
        if ((lane & 7) == 0) yv[pr][8 * h + (lane >> 3)] = tot;
      }
    }
    __syncthreads();
    const int pr = tid % TF_ROWS, c = tid / TF_ROWS;  // c < NB for tid < TF_ROWS NB
    const int p = p0 + pr;
    if (p < Jt && c < nbt) {
      double t = 0.0;
      for (int q = 0; q <= c; ++q) t += yv[pr][q] * tpp[q][c];
      T[p + (int64_t)(Jt + c) * ldt] = -t;
    }
    return;
  }
  const int nb = m - J < NB ? m - J : NB;
  const int rows = L - J;
  const double *Sp = S + J + (int64_t)J * lds;  // Sp[r + q * lds]: panel vector q, row J + r
  if (bid >= ntrail) {
    // ---- X = S_{<J}^t S_p: wave w of workgroup bid - ntrail takes column q
    const int q = (bid - ntrail) * (TR_TPB / 64) + w;
    if (q >= J) return;  // the whole wave (no barrier follows)
    const double *sq = S + (int64_t)q * lds + J;
    double d[NB];
#pragma unroll
    for (int c = 0; c < NB; ++c) d[c] = 0.0;
    for (int r0 = 0; r0 < rows; r0 += 64 * 4) {
      double sv[4], pv[4][NB];
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = r0 + lane + 64 * i, rc = r < rows ? r : rows - 1;
        sv[i] = r < rows ? sq[rc] : 0.0;
#pragma unroll
        for (int c = 0; c < NB; ++c) pv[i][c] = Sp[rc + (int64_t)(c < nb ? c : nb - 1) * lds];
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int c = 0; c < NB; ++c) d[c] += sv[i] * pv[i][c];
    }
#pragma unroll
    for (int h = 0; h < NB / 8; ++h) {
      double v8[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) v8[k] = d[8 * h + k];
      const double tot = wave_sum8(v8);
      const int c = 8 * h + (lane >> 3);
      if ((lane & 7) == 0 && c < nb) Xc[q + (int64_t)c * m] = tot;
    }
    return;
  }
  // ---- trailing column
  const int k = J + nb + bid;
  double *zk = Z + (int64_t)k * ldz + J;
  if (tid < NB * NB) {
    const int q = tid % NB, c = tid / NB;
    tpp[q][c] = (q < nb && c < nb && q <= c) ? T[(J + q) + (int64_t)(J + c) * ldt] : 0.0;
  }
  double zr[RC], d[NB];
#pragma unroll
  for (int q = 0; q < NB; ++q) d[q] = 0.0;
  // clamped row and column indices (every load in bounds, no branches, so
  // the loads issue together); rows beyond the sketch carry z = 0 and
  // columns beyond nb are not used
#pragma unroll
  for (int i = 0; i < RC; ++i) {
    const int r = tid + TR_TPB * i;
    zr[i] = r < rows ? zk[r < rows ? r : rows - 1] : 0.0;
  }
#pragma unroll
  for (int i = 0; i < RC; ++i) {
    const int r = tid + TR_TPB * i, rc = r < rows ? r : rows - 1;
#pragma unroll
    for (int q = 0; q < NB; ++q) d[q] += Sp[rc + (int64_t)(q < nb ? q : nb - 1) * lds] * zr[i];
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
      if (q <= c) t += tpp[q][c] * d[q];
    u[c] = c < nb ? t : 0.0;
  }
#pragma unroll
  for (int i = 0; i < RC; ++i) {
    const int r = tid + TR_TPB * i, rc = r < rows ? r : rows - 1;
    double zv = zr[i];
#pragma unroll
    for (int c = 0; c < NB; ++c)
      if (c < nb) zv -= Sp[rc + (int64_t)c * lds] * u[c];
    if (r < rows) zk[r] = zv;
  }
}

template <int NB>
int hqr_panel_launch(int rpt, int32_t L, int32_t m, int32_t J, double *Zc, double *S, int64_t lds,
                     double *T, int64_t ldt, double *R, int64_t ldr, int32_t *status,
                     hipStream_t st) {
#define RHQR_HQR_PANEL(RPTV)                                                                    \
  case RPTV:                                                                                    \
    RHQR_LAUNCH(RHQR_PROF_HQR, (k_hqr_panel<NB, RPTV>), dim3(1), dim3(HQ_TPB), 0, st, L, m, J,   \
                Zc, (int64_t)L, S, lds, T, ldt, R, ldr, (int)RHQR_SCALE_UNIT_PIVOT, status);   \
    return RHQR_OK
  switch (rpt) {
    RHQR_HQR_PANEL(1);
    RHQR_HQR_PANEL(2);
    RHQR_HQR_PANEL(3);
    RHQR_HQR_PANEL(4);
    RHQR_HQR_PANEL(5);
    RHQR_HQR_PANEL(6);
    RHQR_HQR_PANEL(7);
    RHQR_HQR_PANEL(8);
    default:
      return RHQR_ERR_UNSUPPORTED;
  }
#undef RHQR_HQR_PANEL
}

// the trail launch with rc rows per thread of the trailing columns (1 .. 8)
template <int NB>
int hqr_trail_launch(int rc, int grid, int32_t L, int32_t m, int32_t J, double *Zc,
                     const double *S, int64_t lds, double *T, int64_t ldt, int ntrail, int nx,
                     double *Xc, int32_t Jt, const double *Xt, hipStream_t st) {
#define RHQR_HQR_TRAIL(RCV)                                                                     \
  case RCV:                                                                                     \
    RHQR_LAUNCH(RHQR_PROF_HQR, (k_hqr_trail<NB, RCV>), dim3((unsigned)grid), dim3(TR_TPB), 0, st, \
                L, m, J, Zc, (int64_t)L, S, lds, T, ldt, ntrail, nx, Xc, Jt, Xt);               \
    return RHQR_OK
  static_assert(TR_MAXRC == 8, "one case per row count");
  switch (rc) {
    RHQR_HQR_TRAIL(1);
    RHQR_HQR_TRAIL(2);
    RHQR_HQR_TRAIL(3);
    RHQR_HQR_TRAIL(4);
    RHQR_HQR_TRAIL(5);
    RHQR_HQR_TRAIL(6);
    RHQR_HQR_TRAIL(7);
    RHQR_HQR_TRAIL(8);
    default:
      return RHQR_ERR_UNSUPPORTED;
  }
#undef RHQR_HQR_TRAIL
}

template <int NB>
int hqr_run(int32_t L, int32_t m, double *Zc, double *S, int64_t lds, double *T, int64_t ldt,
            double *R, int64_t ldr, double *X0, double *X1, int32_t *status, hipStream_t st) {
  double *Xb[2] = {X0, X1};
  int32_t Jprev = -1;  // the panel whose block of T is still to be formed
  for (int32_t J = 0; J < m; J += NB) {
    const int32_t nb = m - J < NB ? m - J : NB;
    const int rpt = (L - J + HQ_TPB - 1) / HQ_TPB;
    int rc = hqr_panel_launch<NB>(rpt, L, m, J, Zc, S, lds, T, ldt, R, ldr, status, st);
    if (rc) return rc;
    const int ntrail = m - J - nb;
    const int nx = (J + TR_TPB / 64 - 1) / (TR_TPB / 64);
    const int ntf = Jprev > 0 ? (Jprev + TF_ROWS - 1) / TF_ROWS : 0;
    const int grid = ntrail + nx + ntf;
    if (grid > 0) {
      double *Xc = Xb[(J / NB) & 1];
      const double *Xt = Jprev >= 0 ? Xb[(Jprev / NB) & 1] : X0;
      rc = hqr_trail_launch<NB>((L - J + TR_TPB - 1) / TR_TPB, grid, L, m, J, Zc, S, lds, T, ldt,
                                ntrail, nx, Xc, Jprev > 0 ? Jprev : 0, Xt, st);
      if (rc) return rc;
    }
    Jprev = J;
  }
  // the last panel's block of T
  if (Jprev > 0) {
    const int ntf = (Jprev + TF_ROWS - 1) / TF_ROWS;
    const int rc = hqr_trail_launch<NB>(1, ntf, L, m, Jprev, Zc, S, lds, T, ldt, 0, 0,
                                        Xb[(Jprev / NB) & 1], Jprev,
                                        (const double *)Xb[(Jprev / NB) & 1], st);
    if (rc) return rc;
  }
  return RHQR_OK;
}

}  // namespace

// Sketch-space Householder QR of Z (L x m float64, copied to Zc, which is
// overwritten): S (Householder vectors, unit pivot), T, R.  X0, X1: two
// m x m float64 scratch buffers (the products S_{<J}^t S_p of consecutive
// panels).
int sketch_space_hqr(int32_t L, int32_t m, double *Zc, double *S, int64_t lds, double *T,
                     int64_t ldt, double *R, int64_t ldr, double *X0, double *X1,
                     const LoopWs &w, hipStream_t st) {
  hipLaunchKernelGGL(k_zero_mat, dim3((m + 255) / 256, m), dim3(256), 0, st, T, ldt, m, m);
  RHQR_HIP(hipGetLastError());
  if (L + m <= SQ_MAXL) {  // the panel in registers; two launches per panel
    return hqr_run<8>(L, m, Zc, S, lds, T, ldt, R, ldr, X0, X1, w.status, st);
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
  rc = sketch_space_hqr(L, m, w.Zc, d_S, lds, d_T, ldt, d_R, ldr, w.G, w.M, w.loop, st);
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
