// trimRHQR: randomized reflectors with partial sketching (Sec. 7), the
// left-looking form of Alg. 12 with trimRHVector (Alg. 10).
//
// Omega (l x n) sketches every row, so l may be smaller than m.  Reflector j
// (0-based) uses Psi_j = [I_j 0; 0 Omega_{j:n}] (eq. psij); for u_j, whose
// first j entries vanish, H_j = I - beta u (Omega u)^t [0 Omega_{j:n}].  The
// compact forms (Props. Qbis, Qmbis) are
//     H_1 ... H_m = I - U T ut,   H_m ... H_1 = I - U T~^t ut,
// with ut = ut((Omega U)^t Omega).  Per column j the n-row work is:
//   w~ = w - U_{<j} c,   c = T~^t [ (Omega U)^t Omega w - slt((Omega U)^t Omega) w ]
//   (one streaming pass over the stored columns, every row), the sketch of w~
//   (the one synchronisation), and the store of u_j = alpha w~_{j:} (rows >= j).
// The slt term needs only K = slt((Omega U)^t Omega_{:, <m}) and the first j
// entries of w, since entry (p, i) of slt is <Omega u_p, Omega e_i> for i < p.
// The sketch-space work is float64 in one workgroup; the head rows of U are
// also kept in float64 (Uh) for the T~ recursion.  SRHT only: its columns
// have unit norm, which the elimination of Alg. 10 needs.
#include "engine.h"

#include <cmath>

namespace {

constexpr int TR_TPB = 1024;

// E[k, i] = (Omega e_i)_k = l^-1/2 d_i (-1)^popcount(r_k & i) for the sampled
// rows r_k (natural-order Walsh-Hadamard entries), i < m
__global__ void k_trim_eye(int32_t l, int32_t m, const uint64_t *__restrict__ signs,
                           const int32_t *__restrict__ rows, double *__restrict__ E) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (k >= l || i >= m) return;
  const double s = 1.0 / sqrt((double)l);
  const bool neg_d = (signs[i >> 6] >> (i & 63)) & 1ull;
  const bool neg_h = __popc((unsigned)rows[k] & (unsigned)i) & 1;
  E[k + (int64_t)i * l] = (neg_d != neg_h) ? -s : s;
}

__device__ __forceinline__ double block_sum(double v, double *red) {
  v = wave_sum(v);
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  __syncthreads();
  if (lane == 0) red[w] = v;
  __syncthreads();
  double t = 0.0;
  for (int i = 0; i < (int)(blockDim.x >> 6); ++i) t += red[i];
  return t;
}

// refresh coefficients of column j: a_p = S_p^t z_j - sum_{i < p} K_{p,i} w_i
// (p < j), c = T~_{<j}^t a.  One workgroup.
template <typename ST>
__global__ void __launch_bounds__(TR_TPB) k_trim_coef(int32_t j, int32_t l, int32_t m,
                                                      const double *__restrict__ S,
                                                      const double *__restrict__ Z,
                                                      const double *__restrict__ K,
                                                      const double *__restrict__ Tt,
                                                      const ST *__restrict__ W, int64_t ldw,
                                                      double *__restrict__ c) {
  __shared__ double a[1024];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const double *zj = Z + (int64_t)j * l;
  const ST *wj = W + (int64_t)j * ldw;
  for (int p = w; p < j; p += TR_TPB / 64) {
    double v = 0.0;
    for (int r = lane; r < l; r += 64) v += S[r + (int64_t)p * l] * zj[r];
    for (int i = lane; i < p; i += 64) v -= K[p + (int64_t)i * m] * cvt_in<double>(wj[i]);
    v = wave_sum(v);
    if (lane == 0) a[p] = v;
  }
  __syncthreads();
  for (int p = w; p < j; p += TR_TPB / 64) {
    double v = 0.0;
    for (int q = lane; q <= p; q += 64) v += Tt[q + (int64_t)p * m] * a[q];
    v = wave_sum(v);
    if (lane == 0) c[p] = v;
  }
}

// w_j -= U_{:, <j} c over every row; VEC rows per thread, 8 columns' loads
// issued together
constexpr int TG_TPB = 256, TG_KB = 8;
template <typename ST>
__global__ void __launch_bounds__(TG_TPB) k_trim_refresh(ST *__restrict__ W, int64_t ldw, int64_t n,
                                                         int32_t j, const double *__restrict__ c,
                                                         int aligned) {
  using CT = typename CompT<ST>::type;
  constexpr int VEC = 16 / sizeof(ST);
  const int64_t r0 = ((int64_t)blockIdx.x * TG_TPB + threadIdx.x) * VEC;
  if (r0 >= n) return;
  const bool fast = aligned && r0 + VEC <= n;
  auto load = [&](int p, CT (&x)[VEC]) {
    const ST *col = W + (int64_t)p * ldw + r0;
    if (fast) {
      vload<ST, CT, true>(col, x);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) x[e] = r0 + e < n ? cvt_in<CT>(col[e]) : (CT)0;
    }
  };
  CT acc[VEC];
  load(j, acc);
  int p = 0;
  for (; p + TG_KB <= j; p += TG_KB) {
    CT x[TG_KB][VEC];
#pragma unroll
    for (int u = 0; u < TG_KB; ++u) load(p + u, x[u]);
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < TG_KB; ++u) {
      const CT cu = (CT)c[p + u];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e] -= x[u][e] * cu;
    }
  }
  for (; p < j; ++p) {
    CT x[VEC];
    load(p, x);
    const CT cu = (CT)c[p];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e] -= x[e] * cu;
  }
  ST *out = W + (int64_t)j * ldw + r0;
  if (fast) {
    vstore<ST, CT>(out, acc);
  } else {
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (r0 + e < n) out[e] = cvt_out<ST>((double)acc[e]);
  }
}

// trimRHVector (Alg. 10) and the T, T~, K, R updates of column j, one
// workgroup.  zeta = Omega w~ (w~ the refreshed column in W); Uh holds the
// head rows (< m) of U in float64.  scal[4 j ..]: sigma rho, the multiplier
// alpha of v (u = alpha v), beta.
template <typename ST>
__global__ void __launch_bounds__(TR_TPB) k_trim_vec(
    int32_t j, int32_t l, int32_t m, int scaling, const double *__restrict__ zeta,
    const double *__restrict__ E, const ST *__restrict__ W, int64_t ldw, double *__restrict__ S,
    double *__restrict__ T, int64_t ldt, double *__restrict__ Tt, double *__restrict__ K,
    double *__restrict__ Uh, double *__restrict__ R, int64_t ldr, double *__restrict__ scal,
    int32_t *__restrict__ status) {
  __shared__ double red[TR_TPB / 64];
  __shared__ double hw[1024];  // w~_i, i <= j
  __shared__ double d[1024], dp[1024], g[1024];
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const ST *wj = W + (int64_t)j * ldw;
  for (int i = tid; i <= j; i += TR_TPB) hw[i] = cvt_in<double>(wj[i]);
  __syncthreads();
  // zeta' = Omega w', w' = w~ with its first j entries zeroed; rho = ||zeta'||
  double ss = 0.0;
  for (int k = tid; k < l; k += TR_TPB) {
    double v = zeta[k];
    for (int i = 0; i < j; ++i) v -= hw[i] * E[k + (int64_t)i * l];
    S[k + (int64_t)j * l] = v;  // unscaled for now
    ss += v * v;
  }
  ss = block_sum(ss, red);
  const double wjj = hw[j];
  const double rho = sqrt(ss);
  const double sigma = wjj >= 0.0 ? 1.0 : -1.0;
  const bool nonfinite = !(isfinite(ss) && isfinite(wjj));
  const bool ident = !(rho > 0.0);
  const double sr = sigma * rho;
  // s = Omega v = zeta' + sigma rho Omega e_j, scaled
  double s2 = 0.0;
  for (int k = tid; k < l; k += TR_TPB) {
    const double v = ident ? E[k + (int64_t)j * l] : S[k + (int64_t)j * l] + sr * E[k + (int64_t)j * l];
    S[k + (int64_t)j * l] = v;
    s2 += v * v;
  }
  s2 = block_sum(s2, red);
  double mult, beta;
  if (ident) {
    mult = 1.0;  // u = e_j, s = Omega e_j, beta = 0
    beta = 0.0;
  } else if (scaling == RHQR_SCALE_UNIT_PIVOT) {
    mult = 1.0 / (wjj + sr);
    beta = 2.0 / (s2 * mult * mult);
  } else {
    mult = sqrt(2.0 / s2);
    beta = 1.0;
  }
  if (!ident)
    for (int k = tid; k < l; k += TR_TPB) S[k + (int64_t)j * l] *= mult;
  __syncthreads();
  // d = S_{<j}^t s_j, g_i = (Omega e_i)^t s_j (i < j, also row j of K)
  for (int p = w; p < j; p += TR_TPB / 64) {
    double v = 0.0, u = 0.0;
    for (int k = lane; k < l; k += 64) {
      const double sj = S[k + (int64_t)j * l];
      v += S[k + (int64_t)p * l] * sj;
      u += E[k + (int64_t)p * l] * sj;
    }
    v = wave_sum(v);
    u = wave_sum(u);
    if (lane == 0) {
      d[p] = v;
      g[p] = u;
      K[j + (int64_t)p * m] = u;
    }
  }
  __syncthreads();
  // d'_p = d_p - sum_{p <= i < j} Uh_{i,p} g_i  ([0 Omega_{j:n}] U_{<j})^t s_j
  for (int p = tid; p < j; p += TR_TPB) {
    double v = d[p];
    for (int i = p; i < j; ++i) v -= Uh[i + (int64_t)p * m] * g[i];
    dp[p] = v;
  }
  __syncthreads();
  // T_{p,j} = -beta (T d)_p, T~_{p,j} = -beta (T~ d')_p, one wave per p
  for (int p = w; p < j; p += TR_TPB / 64) {
    double v = 0.0, u = 0.0;
    for (int q = p + lane; q < j; q += 64) {
      v += T[p + (int64_t)q * ldt] * d[q];
      u += Tt[p + (int64_t)q * m] * dp[q];
    }
    v = wave_sum(v);
    u = wave_sum(u);
    if (lane == 0) {
      T[p + (int64_t)j * ldt] = -beta * v;
      Tt[p + (int64_t)j * m] = -beta * u;
    }
  }
  // head rows of u_j (float64), R column j, scalars
  for (int i = tid; i < m; i += TR_TPB) {
    double u = 0.0;
    if (i == j) u = ident ? 1.0 : (wjj + sr) * mult;
    else if (i > j) u = ident ? 0.0 : cvt_in<double>(wj[i]) * mult;
    Uh[i + (int64_t)j * m] = u;
    R[i + (int64_t)j * ldr] = i < j ? hw[i] : (i == j ? -sr : 0.0);
  }
  if (tid == 0) {
    T[j + (int64_t)j * ldt] = beta;
    Tt[j + (int64_t)j * m] = beta;
    scal[4 * j + 0] = sr;
    scal[4 * j + 1] = mult;
    scal[4 * j + 2] = beta;
    scal[4 * j + 3] = ident ? 1.0 : 0.0;
    if (ident) atomicCAS(status, 0, j + 1);
    if (nonfinite) atomicCAS(status + 1, 0, j + 1);
  }
}

// u_j = alpha (0_{j}; w~_j + sigma rho; w~_{j+1:}) in place of column j
template <typename ST>
__global__ void k_trim_store(ST *__restrict__ W, int64_t ldw, int64_t n, int32_t j,
                             const double *__restrict__ scal) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double sr = scal[4 * j], mult = scal[4 * j + 1];
  const bool ident = scal[4 * j + 3] != 0.0;
  ST *col = W + (int64_t)j * ldw;
  double u;
  if (i < j) u = 0.0;
  else if (i == j) u = ident ? 1.0 : (cvt_in<double>(col[i]) + sr) * mult;
  else u = ident ? 0.0 : cvt_in<double>(col[i]) * mult;
  col[i] = cvt_out<ST>(u);
}

// Mq = T G, G_{p,i} = s_p^t Omega e_i for i >= p (the m x m block of
// ut((Omega U)^t Omega) [I_m; 0]); one thread per entry
__global__ void k_trim_mq(int32_t l, int32_t m, const double *__restrict__ S,
                          const double *__restrict__ E, const double *__restrict__ T, int64_t ldt,
                          double *__restrict__ G, double *__restrict__ Mq, int stage) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  const int i = blockIdx.y;
  if (p >= m) return;
  if (stage == 0) {
    double v = 0.0;
    if (i >= p)
      for (int k = 0; k < l; ++k) v += S[k + (int64_t)p * l] * E[k + (int64_t)i * l];
    G[p + (int64_t)i * m] = v;
  } else {
    double v = 0.0;
    for (int q = p; q <= i; ++q) v += T[p + (int64_t)q * ldt] * G[q + (int64_t)i * m];
    Mq[p + (int64_t)i * m] = v;
  }
}

// Q = [I_m; 0] - U Mq, 32 columns of Q per grid row, one row per thread
template <typename ST>
__global__ void __launch_bounds__(256) k_trim_q(int64_t n, int32_t m, const ST *__restrict__ U,
                                                int64_t ldu, const double *__restrict__ Mq,
                                                ST *__restrict__ Q, int64_t ldq) {
  using CT = typename CompT<ST>::type;
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  const int c0 = blockIdx.y * 32;
  if (i >= n) return;
  CT acc[32];
#pragma unroll
  for (int c = 0; c < 32; ++c) acc[c] = (CT)(i == c0 + c ? 1.0 : 0.0);
  for (int p = 0; p < m; ++p) {
    const CT u = cvt_in<CT>(U[i + (int64_t)p * ldu]);
#pragma unroll
    for (int c = 0; c < 32; ++c)
      if (c0 + c < m) acc[c] -= u * (CT)Mq[p + (int64_t)(c0 + c) * m];
  }
#pragma unroll
  for (int c = 0; c < 32; ++c)
    if (c0 + c < m) Q[i + (int64_t)(c0 + c) * ldq] = cvt_out<ST>((double)acc[c]);
}

struct TrimWs {
  int32_t *status;
  double *Z, *E, *K, *Tt, *Uh, *zeta, *c, *scal, *G, *Mq;
  void *skws;
  size_t skws_bytes;
};

size_t trim_ws_bytes(const rhqr_sketch_s *h, int32_t m) {
  const size_t l = h->l;
  size_t b = align_up(sizeof(int32_t) * 4);
  b += 2 * align_up(sizeof(double) * l * m);                // Z, E
  b += 5 * align_up(sizeof(double) * (size_t)m * m);        // K, Tt, Uh, G, Mq
  b += align_up(sizeof(double) * l);                        // zeta
  b += align_up(sizeof(double) * m);                        // c
  b += align_up(sizeof(double) * 4 * m);                    // scal
  size_t sk = sketch_ws_bytes(h, m), s1 = sketch_ws_bytes(h, 1);
  b += align_up(sk > s1 ? sk : s1);
  return b;
}

int trim_ws_carve(const rhqr_sketch_s *h, int32_t m, void *ws, size_t bytes, TrimWs *o) {
  if (bytes < trim_ws_bytes(h, m)) return RHQR_ERR_WORKSPACE;
  const size_t l = h->l;
  char *p = (char *)ws;
  auto take = [&](size_t b) {
    char *r = p;
    p += align_up(b);
    return (void *)r;
  };
  o->status = (int32_t *)take(sizeof(int32_t) * 4);
  o->Z = (double *)take(sizeof(double) * l * m);
  o->E = (double *)take(sizeof(double) * l * m);
  o->K = (double *)take(sizeof(double) * (size_t)m * m);
  o->Tt = (double *)take(sizeof(double) * (size_t)m * m);
  o->Uh = (double *)take(sizeof(double) * (size_t)m * m);
  o->G = (double *)take(sizeof(double) * (size_t)m * m);
  o->Mq = (double *)take(sizeof(double) * (size_t)m * m);
  o->zeta = (double *)take(sizeof(double) * l);
  o->c = (double *)take(sizeof(double) * m);
  o->scal = (double *)take(sizeof(double) * 4 * m);
  size_t sk = sketch_ws_bytes(h, m), s1 = sketch_ws_bytes(h, 1);
  o->skws_bytes = align_up(sk > s1 ? sk : s1);
  o->skws = take(o->skws_bytes);
  return RHQR_OK;
}

__global__ void k_trim_zero(double *p, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0.0;
}

__global__ void k_trim_zero_ld(double *A, int64_t lda, int32_t m) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r < m) A[r + (int64_t)blockIdx.y * lda] = 0.0;
}

template <typename ST>
int trim_typed(const rhqr_sketch_s *h, int64_t n, int32_t m, ST *W, int64_t ldw, double *S,
               double *T, int64_t ldt, double *R, int64_t ldr, ST *Q, int64_t ldq, int scaling,
               const TrimWs &w, hipStream_t st) {
  const int32_t l = h->l;
  const int aligned = ((uintptr_t)W % 16 == 0) && ((ldw * (int64_t)sizeof(ST)) % 16 == 0);
  int rc = launch_fill(w.status, 16, st);
  if (rc) return rc;
  const int64_t mm = (int64_t)m * m;
  hipLaunchKernelGGL(k_trim_zero, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st, w.K, mm);
  hipLaunchKernelGGL(k_trim_zero, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st, w.Tt, mm);
  hipLaunchKernelGGL(k_trim_zero, dim3((unsigned)((mm + 255) / 256)), dim3(256), 0, st, w.Uh, mm);
  hipLaunchKernelGGL(k_trim_zero_ld, dim3((m + 255) / 256, m), dim3(256), 0, st, T, ldt, m);
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_trim_eye, dim3((l + 255) / 256, m), dim3(256), 0, st, l, m, h->d_signs,
                     h->d_rows, w.E);
  RHQR_HIP(hipGetLastError());
  // Omega w_j of every column, taken once up front (Alg. 12 sketches w at the
  // top of each iteration, before it is changed)
  rc = launch_sketch(h, sizeof(ST) == 8 ? RHQR_F64 : RHQR_F32, n, m, W, ldw, w.Z, l, w.skws,
                     w.skws_bytes, st);
  if (rc) return rc;
  const dim3 rgrid((unsigned)((n + (int64_t)TG_TPB * (16 / sizeof(ST)) - 1) /
                              ((int64_t)TG_TPB * (16 / sizeof(ST)))));
  const dim3 sgrid((unsigned)((n + 255) / 256));
  for (int32_t j = 0; j < m; ++j) {
    if (j >= 1) {
      hipLaunchKernelGGL((k_trim_coef<ST>), dim3(1), dim3(TR_TPB), 0, st, j, l, m,
                         (const double *)S, (const double *)w.Z, (const double *)w.K,
                         (const double *)w.Tt, (const ST *)W, ldw, w.c);
      RHQR_HIP(hipGetLastError());
      RHQR_LAUNCH(RHQR_PROF_TALL, (k_trim_refresh<ST>), rgrid, dim3(TG_TPB), 0, st, W, ldw, n, j,
                  (const double *)w.c, aligned);
    }
    rc = launch_sketch(h, sizeof(ST) == 8 ? RHQR_F64 : RHQR_F32, n, 1, W + (int64_t)j * ldw, ldw,
                       w.zeta, l, w.skws, w.skws_bytes, st);
    if (rc) return rc;
    RHQR_LAUNCH(RHQR_PROF_FIN, (k_trim_vec<ST>), dim3(1), dim3(TR_TPB), 0, st, j, l, m, scaling,
                (const double *)w.zeta, (const double *)w.E, (const ST *)W, ldw, S, T, ldt, w.Tt,
                w.K, w.Uh, R, ldr, w.scal, w.status);
    hipLaunchKernelGGL((k_trim_store<ST>), sgrid, dim3(256), 0, st, W, ldw, n, j,
                       (const double *)w.scal);
    RHQR_HIP(hipGetLastError());
  }
  if (Q) {
    hipLaunchKernelGGL(k_trim_mq, dim3((m + 255) / 256, m), dim3(256), 0, st, l, m,
                       (const double *)S, (const double *)w.E, (const double *)T, ldt, w.G, w.Mq,
                       0);
    hipLaunchKernelGGL(k_trim_mq, dim3((m + 255) / 256, m), dim3(256), 0, st, l, m,
                       (const double *)S, (const double *)w.E, (const double *)T, ldt, w.G, w.Mq,
                       1);
    RHQR_HIP(hipGetLastError());
    RHQR_LAUNCH(RHQR_PROF_QTAIL, (k_trim_q<ST>), dim3((unsigned)((n + 255) / 256), (m + 31) / 32),
                dim3(256), 0, st, n, m, (const ST *)W, ldw, (const double *)w.Mq, Q, ldq);
  }
  return RHQR_OK;
}

}  // namespace

extern "C" size_t rhqr_trim_workspace_size(rhqr_sketch_t h, int dtype, int32_t m) {
  if (!h || h->m != 0 || h->kind != RHQR_SKETCH_SRHT || m < 1 || m > 1024 || m > h->n ||
      (dtype != RHQR_F64 && dtype != RHQR_F32))
    return 0;
  return trim_ws_bytes(h, m);
}

extern "C" int rhqr_trim_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W,
                                int64_t ldw, double *d_S, int64_t lds, double *d_T, int64_t ldt,
                                double *d_Tt, int64_t ldtt, double *d_R, int64_t ldr, void *d_Q,
                                int64_t ldq, int opts, void *d_ws, size_t ws_bytes, void *stream) {
  if (!h || h->m != 0 || h->kind != RHQR_SKETCH_SRHT) return -1;
  if (dtype != RHQR_F64 && dtype != RHQR_F32) return -2;
  if (n != h->n) return -3;
  if (m < 1 || m > 1024 || m > n) return -4;
  if (!d_W) return -5;
  if (ldw < n) return -6;
  if (!d_S) return -7;
  if (lds != h->l) return -8;
  if (!d_T) return -9;
  if (ldt < m) return -10;
  if (!d_Tt) return -11;
  if (ldtt < m) return -12;
  if (!d_R) return -13;
  if (ldr < m) return -14;
  if (d_Q && ldq < n) return -16;
  const int scaling = opts & 0xff;
  if ((scaling != RHQR_SCALE_UNIT_PIVOT && scaling != RHQR_SCALE_SQRT2) || (opts >> 8) != 0)
    return -17;
  if (!d_ws) return -18;
  TrimWs w;
  int rc = trim_ws_carve(h, m, d_ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  if (dtype == RHQR_F64)
    rc = trim_typed<double>(h, n, m, (double *)d_W, ldw, d_S, d_T, ldt, d_R, ldr, (double *)d_Q,
                            ldq, scaling, w, st);
  else
    rc = trim_typed<float>(h, n, m, (float *)d_W, ldw, d_S, d_T, ldt, d_R, ldr, (float *)d_Q, ldq,
                           scaling, w, st);
  if (rc) return rc;
  // T~ to the caller's layout
  RHQR_HIP(hipMemcpy2DAsync(d_Tt, (size_t)ldtt * sizeof(double), w.Tt, (size_t)m * sizeof(double),
                            (size_t)m * sizeof(double), (size_t)m, hipMemcpyDeviceToDevice, st));
  return RHQR_OK;
}
