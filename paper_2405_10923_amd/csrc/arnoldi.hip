// RHQR-Arnoldi (Alg. 7): the Arnoldi basis of K(A, r0) kept in the compact
// form of left-looking RHQR, one column per call; plus a float64 CSR sparse
// matrix-vector product for the GMRES workload.
//
// Column j (0-based) of the basis is formed from w = A q_{j-1}:
//   z = Psi w;  c = T_{<j}^t S_{<j}^t z;  w~ = w - U_{<j} c;  z = Psi w~   (Alg. 7)
//   RHVector(w~, z) -> u_j, s_j, T_{:,j};  h_{j-1} = (w~_{1:j}; -sigma rho; 0)
//   q_j = e_j - U_{<=j} T_{<=j} S_{<=j}^t e_j
// The sketch Psi keeps k = mmax + 1 head rows (the loop forms mmax + 1
// reflectors).  The refresh, the re-sketch and the float64 step reuse the
// column engine of left-looking RHQR.
#include "engine.h"

#include <cmath>

constexpr int NORM_BLOCKS = 1024;  // workgroups of the residual-norm reduction

struct rhqr_arnoldi_s {
  rhqr_sketch_s *h;
  int dtype;
  int64_t n;
  int32_t k;   // head rows = capacity in columns (mmax + 1)
  int32_t nc;  // reflectors formed
  void *U;     // n x k, dtype (tail rows of the Householder vectors)
  double *S, *T, *R, *Z, *g, *gf;
  double *Hs;       // k x k: rotated copy of H for the least-squares solve
  double *lsres;    // least-squares residual of the last solve, residual norms
  double *ys;       // k: least-squares solution of the GMRES driver
  double *r64;      // n: float64 residual b - A x (GMRES driver)
  double *npart;    // 2 NORM_BLOCKS partial sums of r^2, b^2 (GMRES driver)
  void *vr, *vq0, *vq1, *vw;  // n each, basis type: residual, q_j, q_{j+1}, A q_j
  void *ws;
  void *vec;
  LoopWs lw;
  void *skws;
  size_t skws_bytes;
  LoopArgs la;
};

namespace {

// partial S_{:,p}^t z over RED_CHUNK rows per workgroup (p < nc), one wave per p
__global__ void __launch_bounds__(1024) k_sdots(int32_t L, int32_t k, int32_t nc,
                                                const double *__restrict__ S, int64_t lds,
                                                const double *__restrict__ z,
                                                double *__restrict__ epart) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int r = (int)blockIdx.x * RED_CHUNK + lane;
  const double zr = r < L ? z[r] : 0.0;
  for (int p = w; p < nc; p += 16) {
    const double v = wave_sum(r < L ? S[r + (int64_t)p * lds] * zr : 0.0);
    if (lane == 0) epart[(int64_t)blockIdx.x * k + p] = v;
  }
}

// c_p = sum_{q <= p} T_{q,p} e_q, e = sum of the partials; cf folds 1/alpha of
// the raw (last formed) column.
__global__ void __launch_bounds__(1024) k_tmv(int32_t k, int32_t nc, int gss,
                                              const double *__restrict__ epart,
                                              const double *__restrict__ T, int64_t ldt,
                                              const double *__restrict__ ia, double *__restrict__ c,
                                              double *__restrict__ cf) {
  __shared__ double e[1024];
  for (int p = threadIdx.x; p < nc; p += blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < gss; ++g) s += epart[(int64_t)g * k + p];
    e[p] = s;
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int p = (int)blockIdx.x * 16 + w;
  if (p >= nc) return;
  double v = 0.0;
  for (int q = lane; q <= p; q += 64) v += T[q + (int64_t)p * ldt] * e[q];
  v = wave_sum(v);
  if (lane == 0) {
    c[p] = v;
    cf[p] = p == nc - 1 ? v * ia[p] : v;
  }
}

// g = T_{<=j} (S_{j, <=j})^t (row j of S is row j of U_1); gf folds 1/alpha_j.
__global__ void k_gvec(int32_t j, const double *__restrict__ T, int64_t ldt,
                       const double *__restrict__ S, int64_t lds, const double *__restrict__ ia,
                       double *__restrict__ g, double *__restrict__ gf) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p > j) return;
  double v = 0.0;
  for (int q = p; q <= j; ++q) v += T[p + (int64_t)q * ldt] * S[j + (int64_t)q * lds];
  g[p] = v;
  gf[p] = p == j ? v * ia[j] : v;
}

// head rows: out_r = a out_r + add_r - sum_{p < ncol} S_{r,p} g_p (float64)
template <typename ST>
__global__ void k_head_comb(int32_t kh, int32_t ncol, const double *__restrict__ S, int64_t lds,
                            const double *__restrict__ g, int unit, int32_t unit_row,
                            const double *__restrict__ yadd, int32_t nadd, int accumulate,
                            ST *__restrict__ out) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= kh) return;
  double v = accumulate ? cvt_in<double>(out[r]) : 0.0;
  if (unit && r == unit_row) v += 1.0;
  if (yadd && r < nadd) v += yadd[r];
  for (int p = 0; p < ncol && p <= r; ++p) v -= S[r + (int64_t)p * lds] * g[p];
  out[r] = cvt_out<ST>(v);
}

// tail rows (i >= kh): out_i = a out_i - sum_{p < ncol} U_{i,p} gf_p (the last
// column may hold the raw refreshed values, in place; gf folds in their
// 1/alpha).  Each thread owns VEC consecutive rows (16-byte loads, eight
// columns' loads issued together) and subtracts the columns in increasing p.
constexpr int GV_TPB = 256, GV_KB = 8;
template <typename ST>
__global__ void __launch_bounds__(GV_TPB) k_tail_gemv(const ST *__restrict__ U, int64_t ldu,
                                                      int64_t n, int32_t kh, int32_t ncol,
                                                      const double *__restrict__ gf,
                                                      int accumulate, ST *__restrict__ out,
                                                      int aligned) {
  using CT = typename CompT<ST>::type;
  constexpr int VEC = 16 / sizeof(ST);
  const int64_t mb = kh - kh % VEC;
  const int64_t r0 = mb + ((int64_t)blockIdx.x * GV_TPB + threadIdx.x) * VEC;
  if (r0 >= n) return;
  const bool fast = aligned && r0 + VEC <= n;
  CT v[VEC];
#pragma unroll
  for (int e = 0; e < VEC; ++e) v[e] = (CT)0;
  if (accumulate) {
    if (fast) {
      vload<ST, CT>(out + r0, v);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[e] = r0 + e < n ? cvt_in<CT>(out[r0 + e]) : (CT)0;
    }
  }
  auto column = [&](int p, CT (&x)[VEC]) {
    const ST *col = U + (int64_t)p * ldu + r0;
    if (fast) {
      vload<ST, CT, true>(col, x);
    } else {
#pragma unroll
      for (int e = 0; e < VEC; ++e) x[e] = r0 + e < n ? cvt_in<CT>(col[e]) : (CT)0;
    }
  };
  int p = 0;
  for (; p + GV_KB <= ncol; p += GV_KB) {
    CT x[GV_KB][VEC];
#pragma unroll
    for (int u = 0; u < GV_KB; ++u) column(p + u, x[u]);
#pragma unroll
    for (int u = 0; u < GV_KB; ++u) {
      const CT g = (CT)gf[p + u];
#pragma unroll
      for (int e = 0; e < VEC; ++e) v[e] -= x[u][e] * g;
    }
  }
  for (; p < ncol; ++p) {
    CT x[VEC];
    column(p, x);
    const CT g = (CT)gf[p];
#pragma unroll
    for (int e = 0; e < VEC; ++e) v[e] -= x[e] * g;
  }
#pragma unroll
  for (int e = 0; e < VEC; ++e)
    if (r0 + e >= kh && r0 + e < n) out[r0 + e] = cvt_out<ST>((double)v[e]);
}

template <typename ST>
void launch_tail_gemv(const ST *U, int64_t ldu, int64_t n, int32_t kh, int32_t ncol,
                      const double *gf, int accumulate, ST *out, hipStream_t st) {
  constexpr int VEC = 16 / sizeof(ST);
  const int aligned = ((uintptr_t)U % 16 == 0) && ((uintptr_t)out % 16 == 0) &&
                      ((ldu * (int64_t)sizeof(ST)) % 16 == 0);
  const int64_t mb = kh - kh % VEC;
  const int64_t threads = (n - mb + VEC - 1) / VEC;
  hipLaunchKernelGGL((k_tail_gemv<ST>), dim3((unsigned)((threads + GV_TPB - 1) / GV_TPB)),
                     dim3(GV_TPB), 0, st, U, ldu, n, kh, ncol, gf, accumulate, out, aligned);
}

// y = A x, A in CSR (float64 values), x and y in the basis type, float64 sums
template <typename ST>
__global__ void k_spmv(int64_t n, const int64_t *__restrict__ ptr, const int32_t *__restrict__ idx,
                       const double *__restrict__ val, const ST *__restrict__ x,
                       ST *__restrict__ y) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) s += val[e] * cvt_in<double>(x[idx[e]]);
  y[i] = cvt_out<ST>(s);
}

template <typename ST>
int q_typed(rhqr_arnoldi_s *a, int32_t j, void *out, hipStream_t st) {
  const int32_t kh = a->k;
  const int32_t L = a->h->l + kh;
  hipLaunchKernelGGL(k_gvec, dim3((j + 1 + 255) / 256), dim3(256), 0, st, j, a->T, (int64_t)kh,
                     a->S, (int64_t)L, a->lw.ia, a->g, a->gf);
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_head_comb<ST>), dim3((kh + 255) / 256), dim3(256), 0, st, kh, j + 1, a->S,
                     (int64_t)L, a->g, 1, j, (const double *)nullptr, 0, 0, (ST *)out);
  RHQR_HIP(hipGetLastError());
  const int64_t nt = a->n - kh;
  if (nt > 0) {
    launch_tail_gemv<ST>((const ST *)a->U, a->n, a->n, kh, j + 1, a->gf, 0, (ST *)out, st);
    RHQR_HIP(hipGetLastError());
  }
  return RHQR_OK;
}

int launch_q(rhqr_arnoldi_s *a, int32_t j, void *out, hipStream_t st) {
  switch (a->dtype) {
    case RHQR_F64: return q_typed<double>(a, j, out, st);
    case RHQR_F32: return q_typed<float>(a, j, out, st);
    case RHQR_F16: return q_typed<__half>(a, j, out, st);
    case RHQR_BF16: return q_typed<__hip_bfloat16>(a, j, out, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

// c = T_{<j}^t S_{<j}^t Z_{:,j}
int launch_coef(rhqr_arnoldi_s *a, int32_t j, hipStream_t st) {
  const int32_t kh = a->k;
  const int32_t L = a->h->l + kh;
  const int gss = (L + RED_CHUNK - 1) / RED_CHUNK;
  hipLaunchKernelGGL(k_sdots, dim3(gss), dim3(1024), 0, st, L, kh, j, a->S, (int64_t)L,
                     a->Z + (int64_t)j * L, a->lw.epart);
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL(k_tmv, dim3((j + 15) / 16), dim3(1024), 0, st, kh, j, gss, a->lw.epart, a->T,
                     (int64_t)kh, a->lw.ia, a->lw.c, a->lw.cf);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

__global__ void k_zero(double *p, int64_t cnt) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < cnt) p[i] = 0.0;
}

}  // namespace

extern "C" int rhqr_arnoldi_create(rhqr_sketch_t h, int dtype, int64_t n, int32_t mmax,
                                   void *stream, rhqr_arnoldi_t *out) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (mmax < 1 || mmax + 1 != h->m || mmax + 1 > 1024) return -4;
  if (!out) return -6;
  hipStream_t st = (hipStream_t)stream;
  rhqr_arnoldi_s *a = new rhqr_arnoldi_s();
  a->h = h;
  a->dtype = dtype;
  a->n = n;
  a->k = mmax + 1;
  a->nc = 0;
  const int32_t kh = a->k, L = h->l + kh;
  const size_t es = dtype_size(dtype);
  const size_t lwb = align_up(loop_ws_bytes(h->kind, dtype, n, kh, h->l));
  a->skws_bytes = align_up(sketch_ws_bytes(h, 1));
  size_t bytes = lwb + a->skws_bytes;
  const size_t offS = bytes;
  bytes += align_up(sizeof(double) * (size_t)L * kh);
  const size_t offT = bytes;
  bytes += align_up(sizeof(double) * (size_t)kh * kh);
  const size_t offR = bytes;
  bytes += align_up(sizeof(double) * (size_t)kh * kh);
  const size_t offZ = bytes;
  bytes += align_up(sizeof(double) * (size_t)L * kh);
  const size_t offg = bytes;
  bytes += 2 * align_up(sizeof(double) * (size_t)kh);
  const size_t offH = bytes;
  bytes += align_up(sizeof(double) * (size_t)kh * kh);
  const size_t offres = bytes;
  bytes += align_up(sizeof(double) * 4);
  const size_t offys = bytes;
  bytes += align_up(sizeof(double) * (size_t)kh);
  const size_t offnp = bytes;
  bytes += align_up(sizeof(double) * 2 * NORM_BLOCKS);  // sums of r^2 and b^2 per workgroup
  if (hipMalloc(&a->ws, bytes) != hipSuccess) {
    delete a;
    return RHQR_ERR_HIP;
  }
  // vectors of the GMRES driver: r (float64) and four basis-type vectors
  const size_t vb = align_up((size_t)n * es);
  if (hipMalloc(&a->vec, align_up(sizeof(double) * (size_t)n) + 4 * vb) != hipSuccess) {
    (void)hipFree(a->ws);
    delete a;
    return RHQR_ERR_HIP;
  }
  if (hipMalloc(&a->U, (size_t)n * kh * es) != hipSuccess) {
    (void)hipFree(a->vec);
    (void)hipFree(a->ws);
    delete a;
    return RHQR_ERR_HIP;
  }
  char *base = (char *)a->ws;
  loop_ws_carve(base, lwb, h->kind, dtype, n, kh, h->l, &a->lw);
  a->skws = base + lwb;
  a->S = (double *)(base + offS);
  a->T = (double *)(base + offT);
  a->R = (double *)(base + offR);
  a->Z = (double *)(base + offZ);
  a->g = (double *)(base + offg);
  a->gf = (double *)(base + offg + align_up(sizeof(double) * (size_t)kh));
  a->Hs = (double *)(base + offH);
  a->lsres = (double *)(base + offres);
  a->ys = (double *)(base + offys);
  a->npart = (double *)(base + offnp);
  char *vbase = (char *)a->vec;
  a->r64 = (double *)vbase;
  vbase += align_up(sizeof(double) * (size_t)n);
  a->vr = vbase;
  a->vq0 = vbase + vb;
  a->vq1 = vbase + 2 * vb;
  a->vw = vbase + 3 * vb;
  LoopArgs &la = a->la;
  la.kind = h->kind;
  la.dtype = dtype;
  la.n = n;
  la.m = kh;
  la.l = h->l;
  la.W = a->U;
  la.ldw = n;
  la.Z = a->Z;
  la.ldz = L;
  la.S = a->S;
  la.lds = L;
  la.T = a->T;
  la.ldt = kh;
  la.R = a->R;
  la.ldr = kh;
  la.scaling = RHQR_SCALE_UNIT_PIVOT;
  la.signs = h->d_signs;
  la.rows = h->d_rows;
  la.omega = h->d_omega;
  la.defer = 0;  // launch_coef forms every coefficient of c
  int rc = launch_fill(a->lw.status, 16, st);
  if (!rc) {
    hipLaunchKernelGGL(k_zero, dim3(((int64_t)kh * kh + 255) / 256), dim3(256), 0, st, a->T,
                       (int64_t)kh * kh);
    if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = RHQR_ERR_HIP;
  }
  if (rc) {
    rhqr_arnoldi_destroy(a);
    return rc;
  }
  *out = a;
  return RHQR_OK;
}

extern "C" int rhqr_arnoldi_destroy(rhqr_arnoldi_t a) {
  if (!a) return -1;
  if (a->U) (void)hipFree(a->U);
  if (a->ws) (void)hipFree(a->ws);
  if (a->vec) (void)hipFree(a->vec);
  delete a;
  return RHQR_OK;
}

extern "C" int rhqr_arnoldi_start(rhqr_arnoldi_t a, const void *d_r0, void *d_q1, double *h_beta,
                                  void *stream) {
  if (!a) return -1;
  if (!d_r0) return -2;
  if (!d_q1) return -3;
  hipStream_t st = (hipStream_t)stream;
  const size_t es = dtype_size(a->dtype);
  const int32_t L = a->h->l + a->k;
  a->nc = 0;
  int rc = launch_fill(a->lw.status, 16, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero, dim3(((int64_t)a->k * a->k + 255) / 256), dim3(256), 0, st, a->T,
                     (int64_t)a->k * a->k);
  RHQR_HIP(hipGetLastError());
  RHQR_HIP(hipMemcpyAsync(a->U, d_r0, (size_t)a->n * es, hipMemcpyDeviceToDevice, st));
  rc = launch_sketch(a->h, a->dtype, a->n, 1, d_r0, a->n, a->Z, L, a->skws, a->skws_bytes, st);
  if (rc) return rc;
  rc = engine_step(a->la, a->lw, 0, 0, st);
  if (rc) return rc;
  rc = launch_q(a, 0, d_q1, st);
  if (rc) return rc;
  a->nc = 1;
  if (h_beta) {
    RHQR_HIP(hipMemcpyAsync(h_beta, a->R, sizeof(double), hipMemcpyDeviceToHost, st));
    RHQR_HIP(hipStreamSynchronize(st));
  }
  return RHQR_OK;
}

extern "C" int rhqr_arnoldi_step(rhqr_arnoldi_t a, const void *d_w, void *d_qnext, double *d_hcol,
                                 void *stream) {
  if (!a) return -1;
  if (!d_w) return -2;
  if (a->nc < 1 || a->nc >= a->k) return -1;
  hipStream_t st = (hipStream_t)stream;
  const int32_t j = a->nc;
  const size_t es = dtype_size(a->dtype);
  const int32_t L = a->h->l + a->k;
  // z = Psi w, c = T^t S^t z, the caller's w becomes column j of the basis
  int rc = launch_sketch(a->h, a->dtype, a->n, 1, d_w, a->n, a->Z + (int64_t)j * L, L, a->skws,
                         a->skws_bytes, st);
  if (rc) return rc;
  rc = launch_coef(a, j, st);
  if (rc) return rc;
  RHQR_HIP(hipMemcpyAsync((char *)a->U + (size_t)j * a->n * es, d_w, (size_t)a->n * es,
                          hipMemcpyDeviceToDevice, st));
  // refresh + re-sketch, then RHVector and the T column in float64
  rc = engine_tall(a->la, a->lw, j, st);
  if (rc) return rc;
  rc = engine_step(a->la, a->lw, j, 0, st);
  if (rc) return rc;
  if (d_hcol)
    RHQR_HIP(hipMemcpyAsync(d_hcol, a->R + (int64_t)j * a->k, sizeof(double) * a->k,
                            hipMemcpyDeviceToDevice, st));
  if (d_qnext) {
    rc = launch_q(a, j, d_qnext, st);
    if (rc) return rc;
  }
  a->nc = j + 1;
  return RHQR_OK;
}

namespace {
// v = T_{<j} (S_{<j,<j})^t y (rows < j of S are rows of U_1)
__global__ void k_solv(int32_t j, const double *__restrict__ T, int64_t ldt,
                       const double *__restrict__ S, int64_t lds, const double *__restrict__ y,
                       double *__restrict__ v) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= j) return;
  double s = 0.0;
  for (int q = p; q < j; ++q) {
    double sy = 0.0;
    for (int r = q; r < j; ++r) sy += S[r + (int64_t)q * lds] * y[r];
    s += T[p + (int64_t)q * ldt] * sy;
  }
  v[p] = s;
}

template <typename ST>
int sol_typed(rhqr_arnoldi_s *a, int32_t j, const double *y, void *x, hipStream_t st) {
  const int32_t kh = a->k;
  const int32_t L = a->h->l + kh;
  hipLaunchKernelGGL(k_solv, dim3((j + 255) / 256), dim3(256), 0, st, j, a->T, (int64_t)kh, a->S,
                     (int64_t)L, y, a->g);
  RHQR_HIP(hipGetLastError());
  // fold 1/alpha of a raw column if it is among the first j (never for j < nc)
  hipLaunchKernelGGL((k_head_comb<ST>), dim3((kh + 255) / 256), dim3(256), 0, st, kh, j, a->S,
                     (int64_t)L, a->g, 0, 0, y, j, 1, (ST *)x);
  RHQR_HIP(hipGetLastError());
  const int64_t nt = a->n - kh;
  if (nt > 0) {
    launch_tail_gemv<ST>((const ST *)a->U, a->n, a->n, kh, j, a->g, 1, (ST *)x, st);
    RHQR_HIP(hipGetLastError());
  }
  return RHQR_OK;
}
}  // namespace

extern "C" int rhqr_arnoldi_solution(rhqr_arnoldi_t a, int32_t j, const double *d_y, void *d_x,
                                     void *stream) {
  if (!a) return -1;
  if (j < 1 || j >= a->nc) return -2;  // columns < j are stored scaled when j < nc
  if (!d_y) return -3;
  if (!d_x) return -4;
  hipStream_t st = (hipStream_t)stream;
  switch (a->dtype) {
    case RHQR_F64: return sol_typed<double>(a, j, d_y, d_x, st);
    case RHQR_F32: return sol_typed<float>(a, j, d_y, d_x, st);
    case RHQR_F16: return sol_typed<__half>(a, j, d_y, d_x, st);
    case RHQR_BF16: return sol_typed<__hip_bfloat16>(a, j, d_y, d_x, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

extern "C" int rhqr_arnoldi_basis(rhqr_arnoldi_t a, void **d_U, double **d_S, double **d_T) {
  if (!a) return -1;
  if (d_U) *d_U = a->U;
  if (d_S) *d_S = a->S;
  if (d_T) *d_T = a->T;
  return RHQR_OK;
}

extern "C" int rhqr_spmv_csr(int dtype, int64_t n, const int64_t *d_ptr, const int32_t *d_idx,
                             const double *d_val, const void *d_x, void *d_y, void *stream) {
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -1;
  if (n < 1) return -2;
  if (!d_ptr) return -3;
  if (!d_idx) return -4;
  if (!d_val) return -5;
  if (!d_x) return -6;
  if (!d_y) return -7;
  hipStream_t st = (hipStream_t)stream;
  dim3 grid((n + 255) / 256);
  switch (dtype) {
    case RHQR_F64: hipLaunchKernelGGL((k_spmv<double>), grid, dim3(256), 0, st, n, d_ptr, d_idx, d_val, (const double *)d_x, (double *)d_y); break;
    case RHQR_F32: hipLaunchKernelGGL((k_spmv<float>), grid, dim3(256), 0, st, n, d_ptr, d_idx, d_val, (const float *)d_x, (float *)d_y); break;
    case RHQR_F16: hipLaunchKernelGGL((k_spmv<__half>), grid, dim3(256), 0, st, n, d_ptr, d_idx, d_val, (const __half *)d_x, (__half *)d_y); break;
    default:
      hipLaunchKernelGGL((k_spmv<__hip_bfloat16>), grid, dim3(256), 0, st, n, d_ptr, d_idx, d_val,
                         (const __hip_bfloat16 *)d_x, (__hip_bfloat16 *)d_y);
  }
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

// ------------------------------------------------ Hessenberg least squares
// min_y || beta e_1 - H y ||_2 for the (j+1) x j upper Hessenberg H whose
// column c is h_{c+1} (the Arnoldi relation A Q_j = Q_{j+1} H) and beta =
// (h_0)_1 = -sigma_1 rho_1: the small least-squares problem of Alg. 8, by
// Givens rotations in float64.  One workgroup: at step i the rotation that
// zeroes H_{i+1,i} is formed, then applied to rows i, i+1 of every later
// column in parallel (columns k > i have had rotations 0..i-1 applied by
// then); back substitution on the rotated triangle, one row per step.
namespace {

constexpr int LS_TPB = 1024;

__global__ void __launch_bounds__(LS_TPB) k_hess_ls(int32_t j, int32_t kh,
                                                    const double *__restrict__ Hcols,
                                                    double *__restrict__ Hs,
                                                    double *__restrict__ y,
                                                    double *__restrict__ res) {
  __shared__ double g[1025];
  __shared__ double rot[2];
  const int t = threadIdx.x;
  // Hs(:, c) = h_{c+1}, rows 0..c+1 (the rest of the column is zero)
  for (int c = t; c < j; c += LS_TPB)
    for (int r = 0; r <= c + 1 && r < kh; ++r)
      Hs[r + (int64_t)c * kh] = Hcols[r + (int64_t)(c + 1) * kh];
  for (int r = t; r <= j; r += LS_TPB) g[r] = r == 0 ? Hcols[0] : 0.0;
  __syncthreads();
  for (int i = 0; i < j; ++i) {
    if (t == 0) {
      const double a = Hs[i + (int64_t)i * kh], b = Hs[i + 1 + (int64_t)i * kh];
      const double r = hypot(a, b);
      const double c = r > 0.0 ? a / r : 1.0, s = r > 0.0 ? b / r : 0.0;
      Hs[i + (int64_t)i * kh] = r;
      Hs[i + 1 + (int64_t)i * kh] = 0.0;
      const double gi = g[i];
      g[i] = c * gi;
      g[i + 1] = -s * gi;
      rot[0] = c;
      rot[1] = s;
    }
    __syncthreads();
    const double c = rot[0], s = rot[1];
    for (int k = i + 1 + t; k < j; k += LS_TPB) {
      double *col = Hs + (int64_t)k * kh;
      const double a = col[i], b = col[i + 1];
      col[i] = c * a + s * b;
      col[i + 1] = -s * a + c * b;
    }
    __syncthreads();
  }
  // R y = g_{0:j}, R = the rotated upper triangle
  for (int i = j - 1; i >= 0; --i) {
    if (t == 0) g[i] = g[i] / Hs[i + (int64_t)i * kh];
    __syncthreads();
    const double yi = g[i];
    for (int k = t; k < i; k += LS_TPB) g[k] -= Hs[k + (int64_t)i * kh] * yi;
    __syncthreads();
  }
  for (int i = t; i < j; i += LS_TPB) y[i] = g[i];
  if (t == 0 && res) *res = fabs(g[j]);
}

// r = b - A x (float64, A in CSR), the residual also rounded to the basis
// type; per-workgroup partial sums of r^2 and of b^2 (grid of NORM_BLOCKS)
template <typename ST>
__global__ void __launch_bounds__(256) k_resid(int64_t n, const int64_t *__restrict__ ptr,
                                               const int32_t *__restrict__ idx,
                                               const double *__restrict__ val,
                                               const double *__restrict__ x,
                                               const double *__restrict__ b,
                                               double *__restrict__ r, ST *__restrict__ rdt,
                                               double *__restrict__ part) {
  double rr = 0.0, bb = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x; i < n; i += (int64_t)gridDim.x * 256) {
    double s = 0.0;
    for (int64_t e = ptr[i]; e < ptr[i + 1]; ++e) s += val[e] * x[idx[e]];
    const double ri = b[i] - s;
    r[i] = ri;
    rdt[i] = cvt_out<ST>(ri);
    rr += ri * ri;
    bb += b[i] * b[i];
  }
  __shared__ double sr[4], sb[4];
  rr = wave_sum(rr);
  bb = wave_sum(bb);
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x >> 6] = rr;
    sb[threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    part[2 * blockIdx.x] = sr[0] + sr[1] + sr[2] + sr[3];
    part[2 * blockIdx.x + 1] = sb[0] + sb[1] + sb[2] + sb[3];
  }
}

// out[0] = sqrt(sum r^2), out[1] = sqrt(sum b^2) over the partials, fixed order
__global__ void __launch_bounds__(256) k_norms(int nb, const double *__restrict__ part,
                                               double *__restrict__ out) {
  double rr = 0.0, bb = 0.0;
  for (int i = threadIdx.x; i < nb; i += 256) {
    rr += part[2 * i];
    bb += part[2 * i + 1];
  }
  __shared__ double sr[4], sb[4];
  rr = wave_sum(rr);
  bb = wave_sum(bb);
  if ((threadIdx.x & 63) == 0) {
    sr[threadIdx.x >> 6] = rr;
    sb[threadIdx.x >> 6] = bb;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    out[0] = sqrt(sr[0] + sr[1] + sr[2] + sr[3]);
    out[1] = sqrt(sb[0] + sb[1] + sb[2] + sb[3]);
  }
}

template <typename ST>
__global__ void k_zero_vec(int64_t n, ST *__restrict__ v) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) v[i] = cvt_out<ST>(0.0);
}

// x += dx (dx in the basis type, x float64)
template <typename ST>
__global__ void k_add64(int64_t n, const ST *__restrict__ dx, double *__restrict__ x) {
  const int64_t i = (int64_t)blockIdx.x * 256 + threadIdx.x;
  if (i < n) x[i] += cvt_in<double>(dx[i]);
}

template <typename ST>
int gmres_typed(rhqr_arnoldi_s *a, const int64_t *ptr, const int32_t *idx, const double *val,
                const double *b, double *x, double tol, int32_t max_cycles, double *h_hist,
                int32_t *h_cycles, int64_t *h_steps, hipStream_t st) {
  const int64_t n = a->n;
  const int32_t m = a->k - 1;
  const dim3 vgrid((unsigned)((n + 255) / 256));
  double nrm[2] = {0.0, 0.0};
  auto residual = [&]() -> int {
    hipLaunchKernelGGL((k_resid<ST>), dim3(NORM_BLOCKS), dim3(256), 0, st, n, ptr, idx, val,
                       (const double *)x, b, a->r64, (ST *)a->vr, a->npart);
    RHQR_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_norms, dim3(1), dim3(256), 0, st, NORM_BLOCKS,
                       (const double *)a->npart, a->lsres + 2);
    RHQR_HIP(hipGetLastError());
    RHQR_HIP(hipMemcpyAsync(nrm, a->lsres + 2, sizeof(nrm), hipMemcpyDeviceToHost, st));
    RHQR_HIP(hipStreamSynchronize(st));
    return RHQR_OK;
  };
  int rc = residual();
  if (rc) return rc;
  const double nb = nrm[1] > 0.0 ? nrm[1] : 1.0;
  int32_t cycles = 0;
  int64_t steps = 0;
  while (cycles < max_cycles) {
    // one cycle of Alg. 8 from r = b - A x, in the basis type
    rc = rhqr_arnoldi_start(a, a->vr, a->vq0, nullptr, st);
    if (rc) return rc;
    void *q = a->vq0, *qn = a->vq1;
    for (int32_t j = 0; j < m; ++j) {
      rc = rhqr_spmv_csr(a->dtype, n, ptr, idx, val, q, a->vw, st);
      if (rc) return rc;
      rc = rhqr_arnoldi_step(a, a->vw, j + 1 < m ? qn : nullptr, nullptr, st);
      if (rc) return rc;
      void *tq = q;
      q = qn;
      qn = tq;
    }
    steps += m;
    hipLaunchKernelGGL(k_hess_ls, dim3(1), dim3(LS_TPB), 0, st, m, a->k, (const double *)a->R,
                       a->Hs, a->ys, a->lsres);
    RHQR_HIP(hipGetLastError());
    // dx = Q_m y in the basis type (a->vw is free now), x += dx in float64
    hipLaunchKernelGGL((k_zero_vec<ST>), vgrid, dim3(256), 0, st, n, (ST *)a->vw);
    RHQR_HIP(hipGetLastError());
    rc = rhqr_arnoldi_solution(a, m, a->ys, a->vw, st);
    if (rc) return rc;
    hipLaunchKernelGGL((k_add64<ST>), vgrid, dim3(256), 0, st, n, (const ST *)a->vw, x);
    RHQR_HIP(hipGetLastError());
    rc = residual();
    if (rc) return rc;
    const double rel = nrm[0] / nb;
    if (h_hist) h_hist[cycles] = rel;
    ++cycles;
    if (rel <= tol) break;
  }
  if (h_cycles) *h_cycles = cycles;
  if (h_steps) *h_steps = steps;
  return RHQR_OK;
}

}  // namespace

extern "C" int rhqr_arnoldi_solve_ls(rhqr_arnoldi_t a, int32_t j, double *d_y, double *d_res,
                                     void *stream) {
  if (!a) return -1;
  if (j < 1 || j >= a->nc) return -2;
  if (!d_y) return -3;
  hipStream_t st = (hipStream_t)stream;
  hipLaunchKernelGGL(k_hess_ls, dim3(1), dim3(LS_TPB), 0, st, j, a->k, (const double *)a->R,
                     a->Hs, d_y, d_res);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

extern "C" int rhqr_gmres_csr(rhqr_arnoldi_t a, const int64_t *d_ptr, const int32_t *d_idx,
                              const double *d_val, const double *d_b, double *d_x, double tol,
                              int32_t max_cycles, double *h_hist, int32_t *h_cycles,
                              int64_t *h_steps, void *stream) {
  if (!a) return -1;
  if (!d_ptr) return -2;
  if (!d_idx) return -3;
  if (!d_val) return -4;
  if (!d_b) return -5;
  if (!d_x) return -6;
  if (!(tol >= 0.0)) return -7;
  if (max_cycles < 1) return -8;
  if (a->k < 2) return -1;
  hipStream_t st = (hipStream_t)stream;
  switch (a->dtype) {
    case RHQR_F64:
      return gmres_typed<double>(a, d_ptr, d_idx, d_val, d_b, d_x, tol, max_cycles, h_hist,
                                 h_cycles, h_steps, st);
    case RHQR_F32:
      return gmres_typed<float>(a, d_ptr, d_idx, d_val, d_b, d_x, tol, max_cycles, h_hist,
                                h_cycles, h_steps, st);
    case RHQR_F16:
      return gmres_typed<__half>(a, d_ptr, d_idx, d_val, d_b, d_x, tol, max_cycles, h_hist,
                                 h_cycles, h_steps, st);
    case RHQR_BF16:
      return gmres_typed<__hip_bfloat16>(a, d_ptr, d_idx, d_val, d_b, d_x, tol, max_cycles, h_hist,
                                         h_cycles, h_steps, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}
