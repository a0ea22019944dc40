// Left-looking RHQR column loop (Alg. 4 with RHVector, Alg. 2) on gfx950.
//
// Per column j (0-based) the n-row work is one streaming pass (k_tall):
//     w~_j = w_j - U_{:, <j} c_j                         (refresh, Alg. 4)
//     u_{j-1} = w~_{j-1} / alpha_{j-1}  stored           (deferred scaling)
//     per-tile partials of Omega w~_j                    (re-sketch)
// followed by three small kernels in float64 (the single synchronisation):
//     k_red : reduce the tile partials to y = Psi w~_j, head rows refreshed
//             in float64 from U_1 = S_{1:m}
//     k_ss  : RHVector scalars (sigma, rho, gamma, beta), s_j, R_{:,j}, and
//             partial dot products S^t s_j and S^t z_{j+1}
//     k_fin : T_{:,j} = -beta T_{j-1} S^t s_j and c_{j+1} = T_j^t S_j^t z_{j+1}
//
// Tall data is column-major in the storage type ST (double, float, half,
// bfloat16); arithmetic on it runs in CT = double for double storage and float
// otherwise.  The raw refreshed column is kept in place, in the storage type,
// until alpha_j is known, and the division by alpha_j is folded into the next
// pass's coefficient.
#include "colstep.h"

#include <hip/hip_ext.h>

#include <algorithm>
#include <atomic>
#include <cmath>
#include <type_traits>
#include <vector>

namespace {


// ----------------------------------------------------- single-problem kernels
template <typename ST, int KIND, int TPW>
__global__ void __launch_bounds__(TALL_TPB) k_tall(const ColProblem P, int32_t j, int32_t p0) {
  tall_block<ST, KIND, TPW>(P, j, p0, blockIdx.x);
}

template <typename ST, int KIND>
__global__ void __launch_bounds__(1024) k_red(const ColProblem P, int32_t j, int next) {
  red_split_block<ST, KIND>(P, j, next, blockIdx.y, blockIdx.x);
}

__global__ void __launch_bounds__(1024) k_fin(const ColProblem P, int32_t j, int next) {
  fin_block(P, j, next, blockIdx.x, gridDim.x);
}

// G = S_{:, <J}^t Z_{:, J:J+nb} (J x nb, ld J), one wave per entry
__global__ void __launch_bounds__(1024) k_pgram(int32_t L, int32_t J, int32_t nb,
                                                const double *__restrict__ S, int64_t lds,
                                                const double *__restrict__ Z, int64_t ldz,
                                                double *__restrict__ G) {
  pgram_block(L, J, nb, S, lds, Z, ldz, G, blockIdx.x);
}

// The same launch with the store of u_{J-1} beside it (the two are
// independent; the panel update after them reads both): workgroups below npg
// form G, the others scale rows of column cidx by 1/alpha, 16 bytes per
// thread (aligned columns; the last rows one by one), as k_scale_col does.
template <typename ST>
__global__ void __launch_bounds__(1024) k_pgram_scale(int32_t L, int32_t J, int32_t nb,
                                                      const double *__restrict__ S, int64_t lds,
                                                      const double *__restrict__ Z, int64_t ldz,
                                                      double *__restrict__ G, int npg,
                                                      ST *__restrict__ W, int64_t ldw, int64_t n,
                                                      int32_t m, int32_t cidx,
                                                      const double *__restrict__ ia) {
  if ((int)blockIdx.x < npg) {
    pgram_block(L, J, nb, S, lds, Z, ldz, G, blockIdx.x);
    return;
  }
  constexpr int VEC = 16 / sizeof(ST);
  ST *col = W + (int64_t)cidx * ldw;
  const double s = ia[cidx];
  const int64_t r0 = m - (m % VEC);  // 16-byte aligned start at or below m
  const int64_t i0 = r0 + ((int64_t)(blockIdx.x - npg) * 1024 + threadIdx.x) * VEC;
  if (i0 >= n) return;
  if (i0 + VEC <= n) {
    ST v[VEC];
    *reinterpret_cast<u32x4 *>(v) = *reinterpret_cast<const u32x4 *>(col + i0);
#pragma unroll
    for (int e = 0; e < VEC; ++e)
      if (i0 + e >= m) v[e] = cvt_out<ST>(cvt_in<double>(v[e]) * s);
    *reinterpret_cast<u32x4 *>(col + i0) = *reinterpret_cast<const u32x4 *>(v);
  } else {
    for (int64_t i = i0; i < n; ++i)
      if (i >= m) col[i] = cvt_out<ST>(cvt_in<double>(col[i]) * s);
  }
}

// rows J0..J-1 of C = T_{<J}^t G, padded to pw entries; grid
// (ceil((J - J0) / PTRI_WAVES), pw), PTRI_WAVES waves per workgroup
__global__ void __launch_bounds__(PTRI_WAVES * 64) k_ptri(int32_t J0, int32_t J, int32_t nb,
                                                         int32_t pw, const double *__restrict__ T,
                                                         int64_t ldt, const double *__restrict__ G,
                                                         double *__restrict__ C) {
  ptri_wave(J0, J, nb, pw, T, ldt, G, C, J0 + blockIdx.x * PTRI_WAVES + (threadIdx.x >> 6),
            blockIdx.y);
}

template <typename ST, int NBC>
__global__ void __launch_bounds__(PANEL_TPB) k_panel(ST *__restrict__ W, int64_t ldw, int64_t n,
                                                     int32_t m, int32_t K0, int32_t J, int32_t nb,
                                                     const double *__restrict__ Ct, int aligned) {
  panel_block<ST, NBC>(W, ldw, n, m, K0, J, nb, Ct, aligned, blockIdx.x, J);
}

// ------------------------------------------------------------ final stores
// Store column cidx (tail rows) as u = raw / alpha; the raw refreshed values
// (the input column itself for cidx == 0) are in place in the storage type.
template <typename ST>
__global__ void k_scale_col(ST *W, int64_t ldw, int64_t n, int32_t m, int32_t cidx,
                            const double *ia) {
  const int64_t i = m + (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  ST *col = W + (int64_t)cidx * ldw;
  col[i] = cvt_out<ST>(cvt_in<double>(col[i]) * ia[cidx]);
}

template <typename ST>
__global__ void k_head_store(ST *W, int64_t ldw, int32_t m, const double *S, int64_t lds) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int cidx = blockIdx.y;
  if (k < m) W[k + (int64_t)cidx * ldw] = cvt_out<ST>(S[k + (int64_t)cidx * lds]);
}

__global__ void k_fill(uint32_t *p, size_t nwords) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nwords) p[i] = 0u;
}

// ----------------------------------------------------------------- thin Q
// Mq = T U_1^t (m x m):  Mq_{p,c} = sum_{q=p..c} T_{p,q} U1_{c,q}
__device__ __forceinline__ void tu1t_entry(int32_t m, const double *T, int64_t ldt, const double *S,
                                           int64_t lds, double *Mq, int p, int cidx) {
  double v = 0.0;
  for (int q = p; q <= cidx; ++q) v += T[p + (int64_t)q * ldt] * S[cidx + (int64_t)q * lds];
  Mq[p + (int64_t)cidx * m] = v;
}

__global__ void k_tu1t(int32_t m, const double *T, int64_t ldt, const double *S, int64_t lds,
                       double *Mq) {
  const int p = blockIdx.x * blockDim.x + threadIdx.x;
  if (p < m) tu1t_entry(m, T, ldt, S, lds, Mq, p, blockIdx.y);
}

// Q head: I - U_1 Mq (float64 U_1 from S)
template <typename ST>
__device__ __forceinline__ void qhead_entry(int32_t m, const double *S, int64_t lds,
                                            const double *Mq, ST *Q, int64_t ldq, int k,
                                            int cidx) {
  double v = (k == cidx) ? 1.0 : 0.0;
  for (int p = 0; p <= k; ++p) v -= S[k + (int64_t)p * lds] * Mq[p + (int64_t)cidx * m];
  Q[k + (int64_t)cidx * ldq] = cvt_out<ST>(v);
}

template <typename ST>
__global__ void k_qhead(int32_t m, const double *S, int64_t lds, const double *Mq, ST *Q,
                        int64_t ldq) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k < m) qhead_entry<ST>(m, S, lds, Mq, Q, ldq, k, blockIdx.y);
}

// ------------------------------------------------------- thin Q, float64
// Q_2 = -U_2 Mq (Mq = T U_1^t, m x m) on float64 matrix cores
// (v_mfma_f64_16x16x4): a workgroup of 4 waves owns 64 rows x QF_NC columns
// of Q_2, each wave 16 rows x QF_NC (QF_NC / 16 accumulator blocks).  The
// 16 x QF_NC slices of Mq are staged in LDS and shared by the waves; every
// lane loads one float64 of U_2 per 4-column step (16 consecutive rows of 4
// columns per wave, 128-byte segments), the next slice's values in flight
// during the products.  Operand layout (probed): A[i = lane % 16][k = lane / 16],
// B[k = lane / 16][j = lane % 16], D[i = lane / 16 + 4 t][j = lane % 16].
constexpr int QF_NC = 128, QF_KC = 16;

__global__ void __launch_bounds__(256) k_qtail64(const double *__restrict__ U, int64_t ldu,
                                                 int64_t rows, int32_t m,
                                                 const double *__restrict__ Mq,
                                                 double *__restrict__ Q, int64_t ldq) {
  __shared__ double Bs[QF_KC][QF_NC + 2];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int64_t r0 = (int64_t)blockIdx.x * 64 + w * 16;  // wave's first row (of U_2 / Q_2)
  const int c0 = blockIdx.y * QF_NC;
  const int i = lane & 15, kq = lane >> 4;
  const int64_t row = r0 + i;
  const bool rok = row < rows;
  f64x4_t acc[QF_NC / 16];
#pragma unroll
  for (int b = 0; b < QF_NC / 16; ++b) acc[b] = f64x4_t{0.0, 0.0, 0.0, 0.0};
  double a[QF_KC / 4];
  auto fetch = [&](int k0) {
#pragma unroll
    for (int s = 0; s < QF_KC / 4; ++s) {
      const int k = k0 + 4 * s + kq;
      a[s] = (rok && k < m) ? U[row + (int64_t)k * ldu] : 0.0;
    }
  };
  fetch(0);
  for (int k0 = 0; k0 < m; k0 += QF_KC) {
    __syncthreads();  // the previous slice has been consumed
    for (int e = threadIdx.x; e < QF_KC * QF_NC; e += 256) {
      const int kk = e / QF_NC, c = e % QF_NC;
      const int k = k0 + kk, col = c0 + c;
      Bs[kk][c] = (k < m && col < m) ? Mq[k + (int64_t)col * m] : 0.0;
    }
    __syncthreads();
    double cur[QF_KC / 4];
#pragma unroll
    for (int s = 0; s < QF_KC / 4; ++s) cur[s] = a[s];
    if (k0 + QF_KC < m) fetch(k0 + QF_KC);
#pragma unroll
    for (int s = 0; s < QF_KC / 4; ++s) {
#pragma unroll
      for (int b = 0; b < QF_NC / 16; ++b)
        acc[b] = __builtin_amdgcn_mfma_f64_16x16x4f64(cur[s], Bs[4 * s + kq][b * 16 + i], acc[b],
                                                      0, 0, 0);
    }
  }
#pragma unroll
  for (int b = 0; b < QF_NC / 16; ++b) {
    const int col = c0 + b * 16 + i;
    if (col >= m) continue;
#pragma unroll
    for (int t = 0; t < 4; ++t) {
      const int64_t r = r0 + kq + 4 * t;
      if (r < rows) Q[r + (int64_t)col * ldq] = -acc[b][t];
    }
  }
}

// C[r0:r1, 0:N2] = alpha * A[r0:r1, 0:K] B  (B float64, K x N2).  64 x 64 tiles,
// 16-deep K steps through LDS, 4 x 4 outputs per thread.
template <typename ST>
__global__ void __launch_bounds__(256) k_gemm_tall(const ST *__restrict__ A, int64_t lda, int64_t r0,
                                                   int64_t r1, int32_t K,
                                                   const double *__restrict__ B, int64_t ldb,
                                                   int32_t N2, ST *__restrict__ C, int64_t ldc,
                                                   double alpha) {
  using CT = typename CompT<ST>::type;
  __shared__ CT As[16][64 + 1];
  __shared__ CT Bs[16][64 + 1];
  const int64_t rb = r0 + (int64_t)blockIdx.x * 64;
  const int cb = blockIdx.y * 64;
  const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
  CT acc[4][4] = {};
  for (int k0 = 0; k0 < K; k0 += 16) {
    __syncthreads();
    for (int e = threadIdx.x; e < 16 * 64; e += 256) {
      const int r = e & 63, kq = e >> 6;
      const int64_t gi = rb + r;
      const int kk = k0 + kq;
      As[kq][r] = (gi < r1 && kk < K) ? cvt_in<CT>(A[gi + (int64_t)kk * lda]) : (CT)0;
      const int kr = e & 15, cc = e >> 4;
      const int kk2 = k0 + kr, col = cb + cc;
      Bs[kr][cc] = (kk2 < K && col < N2) ? (CT)B[kk2 + (int64_t)col * ldb] : (CT)0;
    }
    __syncthreads();
#pragma unroll
    for (int kq = 0; kq < 16; ++kq) {
      CT a[4], b[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) a[i] = As[kq][ty + 16 * i];
#pragma unroll
      for (int jj = 0; jj < 4; ++jj) b[jj] = Bs[kq][tx + 16 * jj];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int jj = 0; jj < 4; ++jj) acc[i][jj] += a[i] * b[jj];
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int jj = 0; jj < 4; ++jj) {
      const int64_t gi = rb + ty + 16 * i;
      const int col = cb + tx + 16 * jj;
      if (gi < r1 && col < N2) C[gi + (int64_t)col * ldc] = cvt_out<ST>((double)(alpha * (double)acc[i][jj]));
    }
}

// ------------------------------------------------------------ host helpers
// Tiles per tall workgroup: about one workgroup per compute unit, at least
// two tiles for 2-byte types (16-byte loads need 8 rows per thread).
// A caller's choice (LoopArgs::tpw: 1, 2 or 4) overrides the default.
inline int tall_tpw(int64_t n, size_t elt, int want = 0) {
  const int64_t ntiles = (n + TILE - 1) / TILE;
  int tpw = want ? want : ntiles >= 1024 ? 4 : ntiles >= 512 ? 2 : 1;
  if (elt == 2 && tpw < 2) tpw = 2;
  return tpw;
}

// e0/e1 non-null: the dispatch itself records the two events (start and end
// of the kernel), as the profiling interface requires
template <typename ST, int KIND, int TPW>
void launch_tall(const ColProblem &P, int32_t j, int32_t p0, hipStream_t st, hipEvent_t e0,
                 hipEvent_t e1) {
  const int64_t rows = (int64_t)TILE * TPW;
  const int64_t g = (P.n + rows - 1) / rows;
  if (e0)
    hipExtLaunchKernelGGL((k_tall<ST, KIND, TPW>), dim3(g), dim3(TALL_TPB), 0, st, e0, e1, 0, P, j,
                          p0);
  else
    hipLaunchKernelGGL((k_tall<ST, KIND, TPW>), dim3(g), dim3(TALL_TPB), 0, st, P, j, p0);
}

template <typename ST, int KIND>
void launch_tall_k(const ColProblem &P, int32_t j, int32_t p0, int tpw, hipStream_t st,
                   hipEvent_t e0, hipEvent_t e1) {
  if constexpr (sizeof(ST) == 2) {
    if (tpw == 4) launch_tall<ST, KIND, 4>(P, j, p0, st, e0, e1);
    else launch_tall<ST, KIND, 2>(P, j, p0, st, e0, e1);
  } else {
    if (tpw == 4) launch_tall<ST, KIND, 4>(P, j, p0, st, e0, e1);
    else if (tpw == 2) launch_tall<ST, KIND, 2>(P, j, p0, st, e0, e1);
    else launch_tall<ST, KIND, 1>(P, j, p0, st, e0, e1);
  }
}

template <typename ST>
int tall_typed(const LoopArgs &a, const LoopWs &w, int32_t j, int32_t p0, hipStream_t st) {
  const int tpw = tall_tpw(a.n, sizeof(ST), a.tpw);
  const ColProblem P = make_col_problem(a, w, tpw);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  if (prof_events(RHQR_PROF_TALL, &e0, &e1)) return RHQR_ERR_HIP;
  switch (a.kind) {
    case RHQR_SKETCH_SRHT: launch_tall_k<ST, RHQR_SKETCH_SRHT>(P, j, p0, tpw, st, e0, e1); break;
    case RHQR_SKETCH_GAUSS: launch_tall_k<ST, RHQR_SKETCH_GAUSS>(P, j, p0, tpw, st, e0, e1); break;
    default: launch_tall_k<ST, RHQR_SKETCH_IDENT>(P, j, p0, tpw, st, e0, e1);
  }
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

template <typename ST>
int step_typed(const LoopArgs &a, const LoopWs &w, int32_t j, int next, hipStream_t st) {
  const ColProblem P = make_col_problem(a, w, tall_tpw(a.n, sizeof(ST), a.tpw));
  if (a.kind == RHQR_SKETCH_IDENT)
    RHQR_LAUNCH(RHQR_PROF_RED, (k_red<ST, RHQR_SKETCH_IDENT>), dim3(red_splits(j), P.gred),
                dim3(1024), 0, st, P, j, next);
  else
    RHQR_LAUNCH(RHQR_PROF_RED, (k_red<ST, RHQR_SKETCH_SRHT>), dim3(red_splits(j), P.gred),
                dim3(1024), 0, st, P, j, next);
  RHQR_LAUNCH(RHQR_PROF_FIN, k_fin, dim3(fin_groups(j)), dim3(1024), 0, st, P, j, next);
  return RHQR_OK;
}

template <typename ST>
int finish_typed(const LoopArgs &a, const LoopWs &w, hipStream_t st) {
  ST *W = (ST *)a.W;
  const int64_t ntail = a.n - a.m;
  if (ntail > 0) {
    hipLaunchKernelGGL((k_scale_col<ST>), dim3((ntail + 255) / 256), dim3(256), 0, st, W, a.ldw,
                       a.n, a.m, a.m - 1, w.ia);
    RHQR_HIP(hipGetLastError());
  }
  hipLaunchKernelGGL((k_head_store<ST>), dim3((a.m + 255) / 256, a.m), dim3(256), 0, st, W, a.ldw,
                     a.m, a.S, a.lds);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

template <typename ST>
int run_typed(const LoopArgs &a, const LoopWs &w, hipStream_t st) {
  for (int32_t j = 0; j < a.m; ++j) {
    if (j >= 1) {
      const int rc = tall_typed<ST>(a, w, j, 0, st);
      if (rc) return rc;
    }
    const int rc = step_typed<ST>(a, w, j, j + 1 < a.m, st);
    if (rc) return rc;
  }
  return finish_typed<ST>(a, w, st);
}

// --------------------------------------------------------- blocked TRSM
// X M = B for n-row B, X (column-major, storage type) and M upper triangular
// (float64), in column blocks of TRSM_NB: for the block starting at J,
//   X_{:, J:J+nb} = (B_{:, J:J+nb} - X_{:, <J} M_{<J, J:J+nb}) M_{J:J+nb, J:J+nb}^{-1}.
// One launch per block: the product streams the solved columns X_{:, <J}
// exactly as the panel update does (eight column loads in flight), then every
// row solves its nb x nb triangle by forward substitution in registers and
// the block is written once.  Rows are independent, so each row's result is
// its own substitution, in float64 (float32 for low precision).
constexpr int TRSM_NB = 16;

// Ct[k * 16 + c] = M[k, J + c] (k < J), Md[p * 16 + c] = M[J + p, J + c]
// (upper triangle of the diagonal block); zero padding beyond nb, ones on the
// padded diagonal.
__global__ void k_trsm_coef(int32_t J, int32_t nb, const double *__restrict__ M, int64_t ldm,
                            double *__restrict__ Ct, double *__restrict__ Md) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k < J) Ct[(int64_t)k * TRSM_NB + c] = c < nb ? M[k + (int64_t)(J + c) * ldm] : 0.0;
  if (k < TRSM_NB) {
    double v = 0.0;
    if (k < nb && c < nb && k <= c) v = M[J + k + (int64_t)(J + c) * ldm];
    if (k == c && c >= nb) v = 1.0;
    Md[k * TRSM_NB + c] = v;
  }
}

// 2-byte storage: the solved columns are also kept in a float32 copy (stage,
// ld = rows) and the product reads that copy, so the substitution carries
// float32 unknowns from block to block as it does inside a block.
template <typename ST>
__global__ void __launch_bounds__(PANEL_TPB) k_trsm_blk(const ST *__restrict__ B, int64_t ldb,
                                                        ST *__restrict__ X, int64_t ldx,
                                                        float *__restrict__ stage,
                                                        int64_t rows, int32_t J, int32_t nb,
                                                        const double *__restrict__ Ct,
                                                        const double *__restrict__ Md,
                                                        int aligned) {
  using CT = typename CompT<ST>::type;
  constexpr bool STG = sizeof(ST) == 2;
  using LT = typename std::conditional<STG, float, ST>::type;  // type the product reads
  constexpr int VEC = sizeof(ST) == 8 ? 2 : 4;
  const int64_t lsg = (rows + 3) & ~(int64_t)3;  // leading dimension of the float32 copy
  const LT *Xr = STG ? (const LT *)stage : (const LT *)X;
  const int64_t ldr = STG ? lsg : ldx;
  constexpr int NBC = TRSM_NB;
  const int64_t rb = (int64_t)blockIdx.x * PANEL_TPB * VEC;
  const int64_t r0 = rb + (int64_t)threadIdx.x * VEC;
  if (r0 >= rows) return;
  const bool fast = aligned && rb + (int64_t)PANEL_TPB * VEC <= rows;  // uniform
  const uint32_t off = (uint32_t)(threadIdx.x * VEC * sizeof(ST));
  CT acc[VEC][NBC];
#pragma unroll
  for (int e = 0; e < VEC; ++e)
#pragma unroll
    for (int c = 0; c < NBC; ++c) acc[e][c] = (CT)0;
  auto coef = [&](int k, int c) -> CT { return (CT)Ct[(int64_t)k * NBC + c]; };
  const uint32_t offr = (uint32_t)(threadIdx.x * VEC * sizeof(LT));
  if (fast) {
    int k = 0;
    for (; k + PANEL_KB <= J; k += PANEL_KB) {
      CT xs[PANEL_KB][VEC];
#pragma unroll
      for (int u = 0; u < PANEL_KB; ++u) {
        const char *cb = (const char *)(Xr + (int64_t)(k + u) * ldr + rb);  // uniform
        panel_load<LT, CT, VEC>((const LT *)(cb + offr), xs[u]);
      }
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
      const char *cb = (const char *)(Xr + (int64_t)k * ldr + rb);
      CT xv[VEC];
      panel_load<LT, CT, VEC>((const LT *)(cb + offr), xv);
#pragma unroll
      for (int c = 0; c < NBC; ++c) {
        const CT ck = coef(k, c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e][c] += xv[e] * ck;
      }
    }
  } else {
    for (int k = 0; k < J; ++k) {
      const LT *col = Xr + (int64_t)k * ldr + r0;
      CT xv[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) xv[e] = r0 + e < rows ? cvt_in<CT>(col[e]) : (CT)0;
#pragma unroll
      for (int c = 0; c < NBC; ++c) {
        const CT ck = coef(k, c);
#pragma unroll
        for (int e = 0; e < VEC; ++e) acc[e][c] += xv[e] * ck;
      }
    }
  }
  // right-hand side of the block, then the block's forward substitution
#pragma unroll
  for (int c = 0; c < NBC; ++c) {
    if (c < nb) {
      const ST *bc = B + (int64_t)(J + c) * ldb + r0;
      CT bv[VEC];
      if (fast) {
        panel_load<ST, CT, VEC>(bc, bv);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e) bv[e] = r0 + e < rows ? cvt_in<CT>(bc[e]) : (CT)0;
      }
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e][c] = bv[e] - acc[e][c];
    }
  }
#pragma unroll
  for (int c = 0; c < NBC; ++c) {
#pragma unroll
    for (int p = 0; p < c; ++p) {
      const CT mpc = (CT)Md[p * NBC + c];
#pragma unroll
      for (int e = 0; e < VEC; ++e) acc[e][c] -= acc[e][p] * mpc;
    }
    const CT d = (CT)Md[c * NBC + c];
#pragma unroll
    for (int e = 0; e < VEC; ++e) acc[e][c] = acc[e][c] / d;
  }
#pragma unroll
  for (int c = 0; c < NBC; ++c) {
    if (c < nb) {
      ST *xc = X + (int64_t)(J + c) * ldx + r0;
      CT xv[VEC];
#pragma unroll
      for (int e = 0; e < VEC; ++e) xv[e] = acc[e][c];
      if (fast) {
        panel_store<ST, CT, VEC>(xc, xv);
        if constexpr (STG)
          *reinterpret_cast<float4 *>(stage + (int64_t)(J + c) * lsg + r0) =
              make_float4(xv[0], xv[1], xv[2], xv[3]);
      } else {
#pragma unroll
        for (int e = 0; e < VEC; ++e)
          if (r0 + e < rows) {
            xc[e] = cvt_out<ST>((double)xv[e]);
            if constexpr (STG) stage[(int64_t)(J + c) * lsg + r0 + e] = (float)xv[e];
          }
      }
    }
  }
}

// ------------------------------- 2-byte products on matrix cores (thin Q)
// Float32-accumulating v_mfma_f32_16x16x32 f16 / bf16 products of n-row data
// with a float64 matrix that is scaled per column by a power of two s_j
// (max |B_{:,j}| / s_j in (1/2, 1]) and split into two storage-type parts,
// B / s = hi + lo, so the coefficients keep about 22 (f16) or 16 (bf16) bits.
// Each wave owns 64 rows: it loads 32 columns with 16-byte row-contiguous
// loads, transposes them through its own LDS slice (the operand needs 8
// consecutive columns per lane) and issues the next chunk's loads before the
// current chunk's products.  Lane L of an operand holds contraction indices
// 8 (L >> 4) .. + 7; the A and B operands use the same assignment, so the
// products do not depend on how the instruction orders them.
constexpr int PM_ROWS = 64;                // rows per wave
constexpr int PM_KC = 32;                  // columns of U per chunk
constexpr int PM_KP = 2 * PM_KC;           // chunks go in pairs; coefficient rows padded to this
constexpr int PM_RS = PM_ROWS + 12;        // LDS stride (elements) of one column slice

typedef _Float16 f16x8_t __attribute__((ext_vector_type(8)));
typedef __bf16 bf16x8_t __attribute__((ext_vector_type(8)));

template <typename ST> __device__ __forceinline__ float dec16(unsigned short b) {
  if constexpr (std::is_same<ST, __half>::value)
    return __half2float(__ushort_as_half(b));
  else
    return __uint_as_float(((uint32_t)b) << 16);
}

template <typename ST>
__device__ __forceinline__ f32x4_t mfma32(const u32x4 a, const u32x4 b, f32x4_t acc) {
  if constexpr (std::is_same<ST, __half>::value)
    return __builtin_amdgcn_mfma_f32_16x16x32_f16(__builtin_bit_cast(f16x8_t, a),
                                                  __builtin_bit_cast(f16x8_t, b), acc, 0, 0, 0);
  else
    return __builtin_amdgcn_mfma_f32_16x16x32_bf16(__builtin_bit_cast(bf16x8_t, a),
                                                   __builtin_bit_cast(bf16x8_t, b), acc, 0, 0, 0);
}

// One wave's 64 rows.  FULL: all rows in bounds and 16-byte aligned; the
// column index of the loads is clamped to J - 1 (finite values, multiplied by
// the zero padding of B), so the loads carry no condition.  !FULL (the last,
// ragged wave): guarded element loads.  Chunks of PM_KC columns go in pairs:
// both chunks' columns and coefficients are loaded first (the first chunk's
// before the second's), so the second chunk's loads are in flight during the
// first chunk's transpose and products, and no load is carried across loop
// iterations.
template <typename ST, bool FULL>
__device__ __forceinline__ void mfma_fetch(const ST *__restrict__ U, int64_t ldu, int64_t n,
                                           int32_t K, int64_t rb, int k0, u32x4 (&buf)[4]) {
  const int lane = threadIdx.x & 63;
  // load lane: column lc (+ 8 r), rows rb + lr .. + 7
  const int lc = lane >> 3, lr = (lane & 7) * 8;
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    const int k = k0 + lc + 8 * r;
    if constexpr (FULL) {
      const int kc = k < K ? k : K - 1;
      buf[r] = vraw_nt(U + (int64_t)kc * ldu + rb + lr);
    } else {
      const ST *src = U + (int64_t)k * ldu + rb + lr;
      unsigned short e[8];
#pragma unroll
      for (int q = 0; q < 8; ++q)
        e[q] = (k < K && rb + lr + q < n) ? __builtin_bit_cast(unsigned short, src[q]) : 0;
      buf[r] = u32x4{(uint32_t)e[0] | ((uint32_t)e[1] << 16), (uint32_t)e[2] | ((uint32_t)e[3] << 16),
                     (uint32_t)e[4] | ((uint32_t)e[5] << 16), (uint32_t)e[6] | ((uint32_t)e[7] << 16)};
    }
  }
}

// the chunk's columns into this wave's LDS slice (column k at sl[k * PM_RS +
// row]), then its products with NC coefficient columns.  The B-operand words
// (8 contraction indices each, hi and lo parts) are in LDS, staged by the
// workgroup: cbh[g * NC + column] for the chunk's 8-row group g.
template <typename ST, int NC>
__device__ __forceinline__ void mfma_chunk(const u32x4 (&buf)[4], const u32x4 *cbh,
                                           const u32x4 *cbl, unsigned short *sl,
                                           f32x4_t (&acc)[4][NC / 16]) {
  static_assert(PM_KC == 32, "one contraction step of 32 columns per chunk");
  const int lane = threadIdx.x & 63;
  const int lc = lane >> 3, lr = (lane & 7) * 8;
  // column starts 8-byte aligned (stride 152 bytes): the four 16-lane groups
  // of an operand read fall in different banks
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    uint2 *d = reinterpret_cast<uint2 *>(sl + (lc + 8 * r) * PM_RS + lr);
    d[0] = uint2{buf[r][0], buf[r][1]};
    d[1] = uint2{buf[r][2], buf[r][3]};
  }
  u32x4 bh[NC / 16], bl[NC / 16];
#pragma unroll
  for (int h = 0; h < NC / 16; ++h) {
    const int o = (lane >> 4) * NC + h * 16 + (lane & 15);
    bh[h] = cbh[o];
    bl[h] = cbl[o];
  }
#pragma unroll
  for (int mb = 0; mb < 4; ++mb) {
    uint32_t a[8];
#pragma unroll
    for (int t = 0; t < 8; ++t) a[t] = sl[(8 * (lane >> 4) + t) * PM_RS + mb * 16 + (lane & 15)];
    const u32x4 av{a[0] | (a[1] << 16), a[2] | (a[3] << 16), a[4] | (a[5] << 16),
                   a[6] | (a[7] << 16)};
#pragma unroll
    for (int h = 0; h < NC / 16; ++h) {
      acc[mb][h] = mfma32<ST>(av, bh[h], acc[mb][h]);
      acc[mb][h] = mfma32<ST>(av, bl[h], acc[mb][h]);
    }
  }
}

// ------------------------------------------------ thin Q, 2-byte storage
// Q_2 = -U_2 Mq on the 16x16x32 f16/bf16 instruction with float32
// accumulation, Mq split per column into a power-of-two scale and hi + lo
// parts in the storage type.  A wave owns 64 rows x QH_NC columns of Q_2
// (4 x QH_NC/16 accumulator blocks) and streams all m columns of U_2 through
// its LDS slice, the second chunk of a pair in flight during the first
// chunk's products.  Tiles of 128 columns: U is read twice at m = 256, and
// each element loaded feeds 256 products (64-column tiles measured 25 %
// slower, and a next-pair prefetch does not fit in registers at this width).
constexpr int QH_NC = 128;

// B operand order for a column tile of QH_NC: row group g (rows 8g..8g+7 of
// Mq), tile column jt: B[((tile * Kg + g) * QH_NC + jt) * 8 + t], Kg = Kp / 8.
// column j of Mq (columns j >= m of the last tile are zero); 256 threads
template <typename ST>
__device__ __forceinline__ void qconv_col(int32_t m, int32_t Kp, const double *__restrict__ Mq,
                                          unsigned short *__restrict__ Bh,
                                          unsigned short *__restrict__ Bl,
                                          float *__restrict__ scale, int j) {
  const bool col = j < m;
  __shared__ float sc;
  double mx = 0.0;
  if (col)
    for (int k = threadIdx.x; k < m; k += blockDim.x) mx = fmax(mx, fabs(Mq[k + (int64_t)j * m]));
  for (int o = 32; o > 0; o >>= 1) mx = fmax(mx, __shfl_xor(mx, o, 64));
  __shared__ double wm[4];
  if ((threadIdx.x & 63) == 0) wm[threadIdx.x >> 6] = mx;
  __syncthreads();
  if (threadIdx.x == 0) {
    const double a = fmax(fmax(wm[0], wm[1]), fmax(wm[2], wm[3]));
    int e = 0;
    if (a > 0.0) (void)frexp(a, &e);
    sc = ldexpf(1.0f, e);
    scale[j] = sc;
  }
  __syncthreads();
  const int tile = j / QH_NC, jt = j % QH_NC, Kg = Kp / 8;
  for (int k = threadIdx.x; k < Kp; k += blockDim.x) {
    const double v = (col && k < m) ? Mq[k + (int64_t)j * m] / (double)sc : 0.0;
    const unsigned short h = enc16<ST>((float)v);
    const unsigned short lo = enc16<ST>((float)(v - (double)dec16<ST>(h)));
    const int64_t o = ((((int64_t)tile * Kg + (k >> 3)) * QH_NC + jt) << 3) + (k & 7);
    Bh[o] = h;
    Bl[o] = lo;
  }
}

template <typename ST>
__global__ void __launch_bounds__(256) k_qconv(int32_t m, int32_t Kp,
                                              const double *__restrict__ Mq,
                                              unsigned short *__restrict__ Bh,
                                              unsigned short *__restrict__ Bl,
                                              float *__restrict__ scale) {
  qconv_col<ST>(m, Kp, Mq, Bh, Bl, scale, blockIdx.x);
}

constexpr int QS_WAVES = 8;  // waves per workgroup of the 2-byte thin Q (64 rows each)

// One wave's 64 rows x one column tile, all m columns of U_2 in chunk pairs.
// The workgroup stages each pair's coefficient words in LDS (double-buffered:
// the next pair's words are loaded during this pair's products and stored
// after them, one barrier per pair), so the 8 waves share one fetch of them.
// Every wave of the workgroup runs the loop (the barriers), `active` ones
// also load and multiply.
template <typename ST, bool FULL>
__device__ __forceinline__ void qtail16_loop(const ST *__restrict__ U, int64_t ldu, int64_t rows,
                                             int32_t m, int32_t Kp, int tile,
                                             const unsigned short *__restrict__ Bh,
                                             const unsigned short *__restrict__ Bl, u32x4 *cb,
                                             unsigned short *sl, int64_t rb, bool active,
                                             f32x4_t (&acc)[4][QH_NC / 16]) {
  constexpr int PART = (PM_KP / 8) * QH_NC;        // words of one part of a pair
  constexpr int CE = 2 * PART / (QS_WAVES * 64);   // words staged per thread and pair
  static_assert(CE * QS_WAVES * 64 == 2 * PART, "staging covers the pair exactly");
  const int Kg = Kp / 8;
  u32x4 cr[CE];
  auto cload = [&](int k0) {
#pragma unroll
    for (int q = 0; q < CE; ++q) {
      const int e = threadIdx.x + q * QS_WAVES * 64;
      const int r = e % PART, g = r / QH_NC, jt = r % QH_NC;
      const unsigned short *B = e < PART ? Bh : Bl;
      cr[q] = *reinterpret_cast<const u32x4 *>(
          B + ((((int64_t)tile * Kg + (k0 >> 3) + g) * QH_NC + jt) << 3));
    }
  };
  auto cstore = [&](int buf) {
#pragma unroll
    for (int q = 0; q < CE; ++q) cb[buf * 2 * PART + threadIdx.x + q * QS_WAVES * 64] = cr[q];
  };
  cload(0);
  cstore(0);
  __syncthreads();
  int buf = 0;
  // chunk pairs as in the panel update (clamped columns times zero
  // coefficients past m)
  for (int k0 = 0; k0 < m; k0 += PM_KP) {
    const bool more = k0 + PM_KP < m;
    if (active) {
      u32x4 ba[4], bb[4];
      mfma_fetch<ST, FULL>(U, ldu, rows, m, rb, k0, ba);
      mfma_fetch<ST, FULL>(U, ldu, rows, m, rb, k0 + PM_KC, bb);
      if (more) cload(k0 + PM_KP);
      const u32x4 *c0 = cb + buf * 2 * PART;
      mfma_chunk<ST, QH_NC>(ba, c0, c0 + PART, sl, acc);
      mfma_chunk<ST, QH_NC>(bb, c0 + 4 * QH_NC, c0 + PART + 4 * QH_NC, sl, acc);
    } else if (more) {
      cload(k0 + PM_KP);
    }
    if (more) cstore(buf ^ 1);
    __syncthreads();
    buf ^= 1;
  }
}

// workgroup `wg` of the 2-byte tail product (one launch: wg = blockIdx.x)
template <typename ST>
__device__ __forceinline__ void qtail16_wg(const ST *__restrict__ U, int64_t ldu, int64_t rows,
                                           int32_t m, int32_t Kp,
                                           const unsigned short *__restrict__ Bh,
                                           const unsigned short *__restrict__ Bl,
                                           const float *__restrict__ scale, ST *__restrict__ Q,
                                           int64_t ldq, int aligned, int tiles, int64_t wg) {
  __shared__ unsigned short lds[QS_WAVES][PM_KC * PM_RS];
  __shared__ u32x4 cb[2 * 2 * (PM_KP / 8) * QH_NC];
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  // workgroup b runs on XCD b % 8: the tiles of one row block go to the same
  // XCD one after another, so U is read from HBM about once
  const int64_t slot = wg >> 3;
  const int tile = (int)(slot % tiles);
  const int64_t blk = (slot / tiles) * 8 + (wg & 7);
  if (blk * QS_WAVES * PM_ROWS >= rows) return;  // the whole workgroup (uniform)
  const int64_t rb = (blk * QS_WAVES + w) * PM_ROWS;
  const bool active = rb < rows;
  const bool full = aligned && rb + PM_ROWS <= rows;
  f32x4_t acc[4][QH_NC / 16];
#pragma unroll
  for (int a = 0; a < 4; ++a)
#pragma unroll
    for (int b = 0; b < QH_NC / 16; ++b) acc[a][b] = f32x4_t{0.f, 0.f, 0.f, 0.f};
  if (full)
    qtail16_loop<ST, true>(U, ldu, rows, m, Kp, tile, Bh, Bl, cb, lds[w], rb, true, acc);
  else
    qtail16_loop<ST, false>(U, ldu, rows, m, Kp, tile, Bh, Bl, cb, lds[w], rb, active, acc);
  if (!active) return;
#pragma unroll
  for (int nb = 0; nb < QH_NC / 16; ++nb) {
    const int col = tile * QH_NC + nb * 16 + (lane & 15);
    if (col >= m) continue;
    const float sj = -scale[col];
    ST *qc = Q + (int64_t)col * ldq;
#pragma unroll
    for (int mb = 0; mb < 4; ++mb) {
      const int64_t r0 = rb + mb * 16 + 4 * (lane >> 4);
      if (full) {
        const uint32_t w0 = (uint32_t)enc16<ST>(sj * acc[mb][nb][0]) |
                            ((uint32_t)enc16<ST>(sj * acc[mb][nb][1]) << 16);
        const uint32_t w1 = (uint32_t)enc16<ST>(sj * acc[mb][nb][2]) |
                            ((uint32_t)enc16<ST>(sj * acc[mb][nb][3]) << 16);
        *reinterpret_cast<uint2 *>(qc + r0) = uint2{w0, w1};
      } else {
#pragma unroll
        for (int t = 0; t < 4; ++t)
          if (r0 + t < rows) qc[r0 + t] = cvt_out<ST>((double)(sj * acc[mb][nb][t]));
      }
    }
  }
}

template <typename ST>
__global__ void __launch_bounds__(QS_WAVES * 64) k_qtail16(const ST *__restrict__ U, int64_t ldu,
                                                           int64_t rows, int32_t m, int32_t Kp,
                                                           const unsigned short *__restrict__ Bh,
                                                           const unsigned short *__restrict__ Bl,
                                                           const float *__restrict__ scale,
                                                           ST *__restrict__ Q, int64_t ldq,
                                                           int aligned, int tiles) {
  qtail16_wg<ST>(U, ldu, rows, m, Kp, Bh, Bl, scale, Q, ldq, aligned, tiles, blockIdx.x);
}


template <typename ST, int NBC>
void launch_panel_w(ST *W, int64_t ldw, int64_t n, int32_t m, int32_t K0, int32_t J, int32_t nb,
                    const double *C, int aligned, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  constexpr int VEC = panel_vec<ST, NBC>();
  const int64_t threads = (n - (m - m % VEC) + VEC - 1) / VEC;
  const dim3 grid((unsigned)((threads + PANEL_TPB - 1) / PANEL_TPB));
  if (e0)
    hipExtLaunchKernelGGL((k_panel<ST, NBC>), grid, dim3(PANEL_TPB), 0, st, e0, e1, 0, W, ldw, n, m,
                          K0, J, nb, C, aligned);
  else
    hipLaunchKernelGGL((k_panel<ST, NBC>), grid, dim3(PANEL_TPB), 0, st, W, ldw, n, m, K0, J, nb,
                       C, aligned);
}

template <typename ST>
void launch_panel(ST *W, int64_t ldw, int64_t n, int32_t m, int32_t K0, int32_t J, int32_t nb,
                  const double *C, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  const int aligned = ((uintptr_t)W % 16 == 0) && ((ldw * (int64_t)sizeof(ST)) % 16 == 0);
  if (nb <= 8)
    launch_panel_w<ST, 8>(W, ldw, n, m, K0, J, nb, C, aligned, st, e0, e1);
  else if (nb <= 16)
    launch_panel_w<ST, 16>(W, ldw, n, m, K0, J, nb, C, aligned, st, e0, e1);
  else
    launch_panel_w<ST, 32>(W, ldw, n, m, K0, J, nb, C, aligned, st, e0, e1);
}

// W[m:n, J:J+nb] -= U[m:n, K0:J] C_{K0:J} on matrix cores (float64 / float32)
template <typename ST, int NC>
__global__ void __launch_bounds__(PX_WAVES * 64, px_min_wg<ST>()) k_panel_mx(ST *__restrict__ W, int64_t ldw,
                                                            int64_t n, int32_t m, int32_t K0,
                                                            int32_t J, int32_t nb, int pw,
                                                            const double *__restrict__ C) {
  panel_mx_block<ST, NC>(W, ldw, W + (int64_t)J * ldw, ldw, false, n, m, K0, J, nb, pw, C,
                         blockIdx.x);
}

template <typename ST, int NC>
int launch_panel_mx(ST *W, int64_t ldw, int64_t n, int32_t m, int32_t K0, int32_t J, int32_t nb,
                    int pw, const double *C, hipStream_t st, hipEvent_t e0, hipEvent_t e1) {
  constexpr int VEC = 16 / sizeof(ST);
  constexpr int WR = px_rg(sizeof(ST)) * 16 * VEC;  // rows per wave
  // the kernel reads NC coefficients per row of C: the caller picks NC = pw >= nb
  if (pw < NC || nb > NC) return RHQR_ERR_UNSUPPORTED;
  const int64_t waves = (n - (m - m % VEC) + WR - 1) / WR;
  const dim3 grid((unsigned)((waves + PX_WAVES - 1) / PX_WAVES));
  if (e0)
    hipExtLaunchKernelGGL((k_panel_mx<ST, NC>), grid, dim3(PX_WAVES * 64), 0, st, e0, e1, 0, W,
                          ldw, n, m, K0, J, nb, pw, C);
  else
    hipLaunchKernelGGL((k_panel_mx<ST, NC>), grid, dim3(PX_WAVES * 64), 0, st, W, ldw, n, m, K0, J,
                       nb, pw, C);
  return RHQR_OK;
}

template <typename ST>
int run_blocked_typed(const LoopArgs &a, const LoopWs &w, int panel, int outer, double *C,
                      double *G, hipStream_t st) {
  ST *W = (ST *)a.W;
  const int32_t m = a.m, L = a.l + a.m;
  const int64_t ntail = a.n - m;
  // W_{:, J:J+nb} -= U_{:, K0:J} C_{K0:J}: finish u_{J-1}, form the
  // coefficients in the sketch space, then one tall product
  const bool colaligned = ((uintptr_t)W % 16 == 0) && ((a.ldw * (int64_t)sizeof(ST)) % 16 == 0);
  auto apply = [&](int32_t K0, int32_t J, int32_t nb) -> int {
    const int64_t ne = (int64_t)J * nb;
    const int npg = (int)((ne + 15) / 16);
    if (ntail > 0 && colaligned) {  // u_{J-1} stored in the coefficient launch
      constexpr int VEC = 16 / sizeof(ST);
      const int64_t r0 = m - (m % VEC);
      const int64_t nsc = (a.n - r0 + 1024LL * VEC - 1) / (1024LL * VEC);
      hipLaunchKernelGGL((k_pgram_scale<ST>), dim3((unsigned)(npg + nsc)), dim3(1024), 0, st, L, J,
                         nb, a.S, a.lds, a.Z, a.ldz, G, npg, W, a.ldw, a.n, m, J - 1, w.ia);
      RHQR_HIP(hipGetLastError());
    } else {
      if (ntail > 0) {
        hipLaunchKernelGGL((k_scale_col<ST>), dim3((ntail + 255) / 256), dim3(256), 0, st, W,
                           a.ldw, a.n, m, J - 1, w.ia);
        RHQR_HIP(hipGetLastError());
      }
      hipLaunchKernelGGL(k_pgram, dim3(npg), dim3(1024), 0, st, L, J, nb, a.S, a.lds, a.Z, a.ldz,
                         G);
      RHQR_HIP(hipGetLastError());
    }
    const int pw = panel_width(nb);
    hipLaunchKernelGGL(k_ptri, dim3((J - K0 + PTRI_WAVES - 1) / PTRI_WAVES, pw),
                       dim3(PTRI_WAVES * 64), 0, st, K0, J, nb, pw, a.T, a.ldt, G, C);
    RHQR_HIP(hipGetLastError());
    if (ntail == 0) return RHQR_OK;
    hipEvent_t e0 = nullptr, e1 = nullptr;
    const int aligned = ((uintptr_t)W % 16 == 0) && ((a.ldw * (int64_t)sizeof(ST)) % 16 == 0);
    const bool mx = aligned && nb > PX_MIN_NB;
    if (prof_events(mx ? RHQR_PROF_PANEL_MX : RHQR_PROF_PANEL_VALU, &e0, &e1)) return RHQR_ERR_HIP;
    int rc = RHQR_OK;
    if (aligned && nb > PX_MIN_NB && nb <= 16) {
      rc = launch_panel_mx<ST, 16>(W, a.ldw, a.n, m, K0, J, nb, pw, (const double *)C, st, e0, e1);
    } else if (aligned && nb > PX_MIN_NB) {
      rc = launch_panel_mx<ST, 32>(W, a.ldw, a.n, m, K0, J, nb, pw, (const double *)C, st, e0, e1);
    } else {  // 8 columns or fewer, or unaligned columns: vector units
      launch_panel<ST>(W, a.ldw, a.n, m, K0, J, nb, (const double *)C, st, e0, e1);
    }
    if (rc) return rc;
    RHQR_HIP(hipGetLastError());
    return RHQR_OK;
  };
  // two levels: outer panels of `outer` columns updated from U_{<J0}, inner
  // panels of `panel` columns from the reflectors of their outer panel only
  if (outer < panel) outer = panel;
  for (int32_t J0 = 0; J0 < m; J0 += outer) {
    const int32_t nbo = m - J0 < outer ? m - J0 : outer;
    if (J0 > 0) {
      const int rc = apply(0, J0, nbo);
      if (rc) return rc;
    }
    for (int32_t J = J0; J < J0 + nbo; J += panel) {
      const int32_t nb = J0 + nbo - J < panel ? J0 + nbo - J : panel;
      if (J > J0) {
        const int rc = apply(J0, J, nb);
        if (rc) return rc;
      }
      for (int32_t j = J; j < J + nb; ++j) {
        if (j >= 1) {
          const int rc = tall_typed<ST>(a, w, j, J, st);
          if (rc) return rc;
        }
        const int rc = step_typed<ST>(a, w, j, j + 1 < m, st);
        if (rc) return rc;
      }
    }
  }
  return finish_typed<ST>(a, w, st);
}

// ------------------------------------------------- block RHQR (Alg. 5)
// Before block J (columns J .. J+nb-1) is factored, every earlier block K
// (columns K .. K+kb-1) is applied to it in turn after a fresh sketch of the
// block:  Y = Psi M,  C = T_KK^t S_K^t Y,  M -= U_K C,  with T_KK the
// diagonal block of T (the block's own T factor).  Then the block goes
// through Alg. 4 with refresh coefficients over its own reflectors only
// (LoopArgs::c0 = J) and its own fresh sketch as the pre-sketch.  The head
// rows of M are updated in float64 from the head rows of U (= those of S) and
// kept in place in W (rounded to the storage type), so the sketches and the
// column loop see the current block.

// G = S_{:, K:K+kb}^t Z_{:, J:J+nb} (kb x nb, ld kb), one wave per entry
__global__ void __launch_bounds__(256) k_a5_gram(int32_t L, int32_t K, int32_t kb, int32_t J,
                                                 int32_t nb, const double *__restrict__ S,
                                                 int64_t lds, const double *__restrict__ Z,
                                                 int64_t ldz, double *__restrict__ G) {
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int e = blockIdx.x * 4 + w;
  if (e >= kb * nb) return;  // uniform across the wave
  const int q = e % kb, c = e / kb;
  const double *sp = S + (int64_t)(K + q) * lds;
  const double *zp = Z + (int64_t)(J + c) * ldz;
  double v = 0.0;
  for (int r = lane; r < L; r += 64) v += sp[r] * zp[r];
  v = wave_sum(v);
  if (lane == 0) G[q + (int64_t)c * kb] = v;
}

// C_{K+p, c} = sum_{q <= p} T_{K+q, K+p} G_{q, c} (row K+p at C + (K+p) pw,
// zero for c >= nb), one thread per entry
__global__ void k_a5_coef(int32_t K, int32_t kb, int32_t nb, int32_t pw,
                          const double *__restrict__ T, int64_t ldt, const double *__restrict__ G,
                          double *__restrict__ C) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= kb * pw) return;
  const int p = e / pw, c = e % pw;
  double v = 0.0;
  if (c < nb)
    for (int q = 0; q <= p; ++q) v += T[(K + q) + (int64_t)(K + p) * ldt] * G[q + (int64_t)c * kb];
  C[(int64_t)(K + p) * pw + c] = v;
}

// head rows of the block: W_{k, J+c} -= sum_p S_{k, K+p} C_{K+p, c}, k < m
template <typename ST>
__global__ void k_a5_head(int32_t m, int32_t K, int32_t kb, int32_t J, int32_t nb, int32_t pw,
                          const double *__restrict__ S, int64_t lds, const double *__restrict__ C,
                          ST *__restrict__ W, int64_t ldw) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (k >= m || c >= nb) return;
  ST *wp = W + k + (int64_t)(J + c) * ldw;
  double v = cvt_in<double>(*wp);
  for (int p = 0; p < kb; ++p) v -= S[k + (int64_t)(K + p) * lds] * C[(int64_t)(K + p) * pw + c];
  *wp = cvt_out<ST>(v);
}

// W[m:n, J:J+nb] -= U[m:n, K:K+kb] C_{K:K+kb}: matrix cores, or vector units
template <typename ST, int NC>
__global__ void __launch_bounds__(PX_WAVES * 64, px_min_wg<ST>()) k_a5_panel_mx(ST *__restrict__ W, int64_t ldw,
                                                               int64_t n, int32_t m, int32_t K,
                                                               int32_t kb, int32_t J, int32_t nb,
                                                               int pw,
                                                               const double *__restrict__ C) {
  panel_mx_block<ST, NC>(W, ldw, W + (int64_t)J * ldw, ldw, false, n, m, K, K + kb, nb, pw, C,
                         blockIdx.x);
}

template <typename ST, int NBC>
__global__ void __launch_bounds__(PANEL_TPB) k_a5_panel(ST *__restrict__ W, int64_t ldw, int64_t n,
                                                        int32_t m, int32_t K, int32_t kb,
                                                        int32_t J, int32_t nb,
                                                        const double *__restrict__ C,
                                                        int aligned) {
  panel_block<ST, NBC>(W, ldw, n, m, K, K + kb, nb, C, aligned, blockIdx.x, J);
}

template <typename ST>
int a5_update(ST *W, int64_t ldw, int64_t n, int32_t m, int32_t K, int32_t kb, int32_t J,
              int32_t nb, int pw, const double *C, hipStream_t st) {
  const int aligned = ((uintptr_t)W % 16 == 0) && ((ldw * (int64_t)sizeof(ST)) % 16 == 0);
  hipEvent_t e0 = nullptr, e1 = nullptr;
  const bool mx = aligned && nb > PX_MIN_NB;
  if (prof_events(mx ? RHQR_PROF_PANEL_MX : RHQR_PROF_PANEL_VALU, &e0, &e1)) return RHQR_ERR_HIP;
  if (mx) {
    constexpr int VEC = 16 / sizeof(ST);
    constexpr int WR = px_rg(sizeof(ST)) * 16 * VEC;
    const int64_t waves = (n - (m - m % VEC) + WR - 1) / WR;
    const dim3 grid((unsigned)((waves + PX_WAVES - 1) / PX_WAVES));
#define RHQR_A5_MX(NC)                                                                      \
  if (e0)                                                                                   \
    hipExtLaunchKernelGGL((k_a5_panel_mx<ST, NC>), grid, dim3(PX_WAVES * 64), 0, st, e0, e1, \
                          0, W, ldw, n, m, K, kb, J, nb, pw, C);                            \
  else                                                                                      \
    hipLaunchKernelGGL((k_a5_panel_mx<ST, NC>), grid, dim3(PX_WAVES * 64), 0, st, W, ldw, n, \
                       m, K, kb, J, nb, pw, C)
    if (pw <= 16) {
      RHQR_A5_MX(16);
    } else {
      RHQR_A5_MX(32);
    }
#undef RHQR_A5_MX
  } else {
#define RHQR_A5_VALU(NBC)                                                                     \
  do {                                                                                        \
    constexpr int VEC = panel_vec<ST, NBC>();                                                 \
    const int64_t threads = (n - (m - m % VEC) + VEC - 1) / VEC;                              \
    const dim3 grid((unsigned)((threads + PANEL_TPB - 1) / PANEL_TPB));                       \
    if (e0)                                                                                   \
      hipExtLaunchKernelGGL((k_a5_panel<ST, NBC>), grid, dim3(PANEL_TPB), 0, st, e0, e1, 0, W, \
                            ldw, n, m, K, kb, J, nb, C, aligned);                             \
    else                                                                                      \
      hipLaunchKernelGGL((k_a5_panel<ST, NBC>), grid, dim3(PANEL_TPB), 0, st, W, ldw, n, m, K, \
                         kb, J, nb, C, aligned);                                              \
  } while (0)
    if (pw <= 8)
      RHQR_A5_VALU(8);
    else if (pw <= 16)
      RHQR_A5_VALU(16);
    else
      RHQR_A5_VALU(32);
#undef RHQR_A5_VALU
  }
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

template <typename ST>
int run_alg5_typed(const rhqr_sketch_s *h, LoopArgs a, const LoopWs &w, int b, double *C,
                   double *G, double *Z, void *skws, size_t skws_bytes, hipStream_t st) {
  ST *W = (ST *)a.W;
  const int32_t m = a.m, L = a.l + a.m;
  const int64_t n = a.n, ntail = n - m;
  a.Z = Z;
  a.ldz = L;
  for (int32_t J = 0; J < m; J += b) {
    const int32_t nb = m - J < b ? m - J : b;
    const int pw = panel_width(nb);
    if (J > 0 && ntail > 0) {  // u_{J-1} is still raw: store it scaled before it is applied
      hipLaunchKernelGGL((k_scale_col<ST>), dim3((ntail + 255) / 256), dim3(256), 0, st, W, a.ldw,
                         n, m, J - 1, w.ia);
      RHQR_HIP(hipGetLastError());
    }
    for (int32_t K = 0; K < J; K += b) {
      const int32_t kb = J - K < b ? J - K : b;
      int rc = launch_sketch(h, a.dtype, n, nb, W + (int64_t)J * a.ldw, a.ldw,
                             Z + (int64_t)J * L, L, skws, skws_bytes, st);
      if (rc) return rc;
      hipLaunchKernelGGL(k_a5_gram, dim3((kb * nb + 3) / 4), dim3(256), 0, st, L, K, kb, J, nb,
                         (const double *)a.S, a.lds, (const double *)Z, (int64_t)L, G);
      RHQR_HIP(hipGetLastError());
      hipLaunchKernelGGL(k_a5_coef, dim3((kb * pw + 255) / 256), dim3(256), 0, st, K, kb, nb, pw,
                         (const double *)a.T, a.ldt, (const double *)G, C);
      RHQR_HIP(hipGetLastError());
      hipLaunchKernelGGL((k_a5_head<ST>), dim3((m + 255) / 256, nb), dim3(256), 0, st, m, K, kb,
                         J, nb, pw, (const double *)a.S, a.lds, (const double *)C, W, a.ldw);
      RHQR_HIP(hipGetLastError());
      if (ntail > 0) {
        rc = a5_update<ST>(W, a.ldw, n, m, K, kb, J, nb, pw, C, st);
        if (rc) return rc;
      }
    }
    // the block's own pre-sketch, then Alg. 4 over its columns
    int rc = launch_sketch(h, a.dtype, n, nb, W + (int64_t)J * a.ldw, a.ldw, Z + (int64_t)J * L,
                           L, skws, skws_bytes, st);
    if (rc) return rc;
    a.c0 = J;
    for (int32_t j = J; j < J + nb; ++j) {
      if (j >= 1) {
        rc = tall_typed<ST>(a, w, j, J, st);
        if (rc) return rc;
      }
      rc = step_typed<ST>(a, w, j, j + 1 < J + nb, st);
      if (rc) return rc;
    }
  }
  return finish_typed<ST>(a, w, st);
}

// ------------------------------------------- thin Q tail on matrix cores
// Q_2 = -U_2 Mq as the panel product with a zero start (panel_mx_block),
// one grid row per QX_NC columns of Q.  k_mqt lays Mq out for it: tile t
// holds Mq[k][t QX_NC + c] at Ct[(t m + k) QX_NC + c], zero beyond column m.
constexpr int QX_NC = 64;

__device__ __forceinline__ void mqt_entry(int32_t m, const double *__restrict__ Mq,
                                          double *__restrict__ Ct, int e, int tile) {
  const int k = e / QX_NC, c = e % QX_NC;
  const int col = tile * QX_NC + c;
  Ct[((int64_t)tile * m + k) * QX_NC + c] = col < m ? Mq[k + (int64_t)col * m] : 0.0;
}

__global__ void k_mqt(int32_t m, const double *__restrict__ Mq, double *__restrict__ Ct) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < m * QX_NC) mqt_entry(m, Mq, Ct, e, blockIdx.y);
}

// workgroup `wg` of the tail product (one launch: wg = blockIdx.x)
template <typename ST>
__device__ __forceinline__ void qtail_mx_wg(int64_t n, int32_t m, const ST *__restrict__ U,
                                            int64_t ldu, const double *__restrict__ Ct,
                                            ST *__restrict__ Q, int64_t ldq, int64_t groups,
                                            int tiles, int64_t wg) {
  // workgroup b runs on XCD b % 8: the tiles of one row group go to the same
  // XCD one after another, so U is read from HBM about once
  const int64_t slot = wg >> 3;
  const int tile = (int)(slot % tiles);
  const int64_t g = (slot / tiles) * 8 + (wg & 7);
  if (g >= groups) return;
  const int c0 = tile * QX_NC;
  const int nb = m - c0 < QX_NC ? m - c0 : QX_NC;
  panel_mx_block<ST, QX_NC>(U, ldu, Q + (int64_t)c0 * ldq, ldq, true, n, m, 0, m, nb, QX_NC,
                            Ct + (int64_t)tile * m * QX_NC, g);
}

template <typename ST>
__global__ void __launch_bounds__(PX_WAVES * 64) k_qtail_mx(int64_t n, int32_t m,
                                                            const ST *__restrict__ U, int64_t ldu,
                                                            const double *__restrict__ Ct,
                                                            ST *__restrict__ Q, int64_t ldq,
                                                            int64_t groups, int tiles) {
  qtail_mx_wg<ST>(n, m, U, ldu, Ct, Q, ldq, groups, tiles, blockIdx.x);
}

template <typename ST>
int thin_q_typed(int64_t n, int32_t m, const ST *U, int64_t ldu, const double *S, int64_t lds,
                 const double *T, int64_t ldt, double *Mq, void *qmf, ST *Q, int64_t ldq,
                 hipStream_t st) {
  hipLaunchKernelGGL(k_tu1t, dim3((m + 255) / 256, m), dim3(256), 0, st, m, T, ldt, S, lds, Mq);
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL((k_qhead<ST>), dim3((m + 255) / 256, m), dim3(256), 0, st, m, S, lds, Mq, Q,
                     ldq);
  RHQR_HIP(hipGetLastError());
  const int64_t rows = n - m;
  // float64 and float32 with 16-byte aligned columns: the matrix-core panel
  // product (for 2-byte storage, re-reading U once per 64 columns of Q costs
  // more than the split-coefficient product below saves)
  if constexpr (sizeof(ST) >= 4) {
    const bool aligned = ((uintptr_t)U % 16 == 0) && ((uintptr_t)Q % 16 == 0) &&
                         ((ldu * (int64_t)sizeof(ST)) % 16 == 0) &&
                         ((ldq * (int64_t)sizeof(ST)) % 16 == 0);
    if (rows > 0 && aligned) {
      const int tiles = (m + QX_NC - 1) / QX_NC;
      double *Ct = (double *)qmf;
      hipLaunchKernelGGL(k_mqt, dim3((m * QX_NC + 255) / 256, tiles), dim3(256), 0, st, m,
                         (const double *)Mq, Ct);
      RHQR_HIP(hipGetLastError());
      const int64_t groups = panel_mx_groups(n, m, (int)sizeof(ST));
      const dim3 grid((unsigned)((groups + 7) / 8 * 8 * tiles));
      RHQR_LAUNCH(RHQR_PROF_QTAIL, (k_qtail_mx<ST>), grid, dim3(PX_WAVES * 64), 0, st, n, m, U,
                  ldu, (const double *)Ct, Q, ldq, groups, tiles);
      return RHQR_OK;
    }
  }
  if (rows > 0) {
    if constexpr (std::is_same<ST, double>::value) {
      dim3 grid((unsigned)((rows + 63) / 64), (m + QF_NC - 1) / QF_NC);
      RHQR_LAUNCH(RHQR_PROF_QTAIL, k_qtail64, grid, dim3(256), 0, st, U + m, ldu, rows, m,
                  (const double *)Mq, Q + m, ldq);
    } else if constexpr (sizeof(ST) == 2) {
      const int Kp = (m + PM_KP - 1) / PM_KP * PM_KP;
      const int tiles = (m + QH_NC - 1) / QH_NC;
      unsigned short *Bh = (unsigned short *)qmf;
      unsigned short *Bl = Bh + (size_t)tiles * Kp * QH_NC;
      float *sc = (float *)(Bl + (size_t)tiles * Kp * QH_NC);
      hipLaunchKernelGGL((k_qconv<ST>), dim3(tiles * QH_NC), dim3(256), 0, st, m, Kp,
                         (const double *)Mq, Bh, Bl, sc);
      RHQR_HIP(hipGetLastError());
      const int aligned = ((uintptr_t)(U + m) % 16 == 0) && ((uintptr_t)(Q + m) % 8 == 0) &&
                          ((ldu * (int64_t)sizeof(ST)) % 16 == 0) &&
                          ((ldq * (int64_t)sizeof(ST)) % 8 == 0);
      const int64_t waves = (rows + PM_ROWS - 1) / PM_ROWS;
      const int64_t blks = (waves + QS_WAVES - 1) / QS_WAVES;
      const dim3 grid((unsigned)((blks + 7) / 8 * 8 * tiles));
      RHQR_LAUNCH(RHQR_PROF_QTAIL, (k_qtail16<ST>), grid, dim3(QS_WAVES * 64), 0, st, U + m, ldu,
                  rows, m, Kp, (const unsigned short *)Bh, (const unsigned short *)Bl,
                  (const float *)sc, Q + m, ldq, aligned, tiles);
    } else {
      dim3 grid((rows + 63) / 64, (m + 63) / 64);
      RHQR_LAUNCH(RHQR_PROF_QTAIL, (k_gemm_tall<ST>), grid, dim3(256), 0, st, U, ldu, (int64_t)m,
                  n, m, (const double *)Mq, (int64_t)m, m, Q, ldq, -1.0);
    }
    RHQR_HIP(hipGetLastError());
  }
  return RHQR_OK;
}

// ------------------------------------------------- thin Q over a batch
// The thin-Q stages of many problems, one launch per stage: the same device
// code per entry and per tail workgroup as thin_q_typed (so every Q equals
// the single-problem one bitwise), each workgroup reading its problem from a
// job table (a skipped problem has m = 0 and tiles = 0).
__global__ void __launch_bounds__(256) kq_tu1t(const ThinQJob *__restrict__ J) {
  const ThinQJob &q = J[blockIdx.x];
  const int cidx = blockIdx.y;
  if (cidx >= q.m) return;
  for (int p = threadIdx.x; p < q.m; p += blockDim.x)
    tu1t_entry(q.m, q.T, q.ldt, q.S, q.lds, q.Mq, p, cidx);
}

template <typename ST>
__global__ void __launch_bounds__(256) kq_qhead(const ThinQJob *__restrict__ J) {
  const ThinQJob &q = J[blockIdx.x];
  const int cidx = blockIdx.y;
  if (cidx >= q.m) return;
  for (int k = threadIdx.x; k < q.m; k += blockDim.x)
    qhead_entry<ST>(q.m, q.S, q.lds, q.Mq, (ST *)q.Q, q.ldq, k, cidx);
}

__global__ void __launch_bounds__(256) kq_mqt(const ThinQJob *__restrict__ J) {
  const ThinQJob &q = J[blockIdx.x];
  const int tile = blockIdx.y;
  if (tile >= q.tiles) return;
  for (int e = blockIdx.z * blockDim.x + threadIdx.x; e < q.m * QX_NC; e += gridDim.z * blockDim.x)
    mqt_entry(q.m, q.Mq, (double *)q.qmf, e, tile);
}

template <typename ST>
__global__ void __launch_bounds__(PX_WAVES * 64) kq_qtail_mx(const ThinQJob *__restrict__ J,
                                                             const ThinQBlock *__restrict__ map) {
  const ThinQBlock b = map[blockIdx.x];
  const ThinQJob &q = J[b.p];
  if (q.m == 0) return;
  qtail_mx_wg<ST>(q.n, q.m, (const ST *)q.U, q.ldu, (const double *)q.qmf, (ST *)q.Q, q.ldq,
                  q.groups, q.tiles, b.local);
}

// split coefficients of a problem's qmf scratch, as thin_q_typed lays them out
struct SplitCoef {
  unsigned short *Bh, *Bl;
  float *sc;
};
__device__ __forceinline__ SplitCoef split_coef(const ThinQJob &q) {
  unsigned short *Bh = (unsigned short *)q.qmf;
  unsigned short *Bl = Bh + (size_t)q.tiles * q.Kp * QH_NC;
  return SplitCoef{Bh, Bl, (float *)(Bl + (size_t)q.tiles * q.Kp * QH_NC)};
}

template <typename ST>
__global__ void __launch_bounds__(256) kq_qconv(const ThinQJob *__restrict__ J) {
  const ThinQJob &q = J[blockIdx.x];
  const int j = blockIdx.y;
  if (q.m == 0 || j >= q.tiles * QH_NC) return;  // the whole workgroup
  const SplitCoef c = split_coef(q);
  qconv_col<ST>(q.m, q.Kp, q.Mq, c.Bh, c.Bl, c.sc, j);
}

template <typename ST>
__global__ void __launch_bounds__(QS_WAVES * 64) kq_qtail16(const ThinQJob *__restrict__ J,
                                                            const ThinQBlock *__restrict__ map) {
  const ThinQBlock b = map[blockIdx.x];
  const ThinQJob &q = J[b.p];
  if (q.m == 0) return;  // the whole workgroup
  const SplitCoef c = split_coef(q);
  qtail16_wg<ST>((const ST *)q.U + q.m, q.ldu, q.n - q.m, q.m, q.Kp, c.Bh, c.Bl, c.sc,
                 (ST *)q.Q + q.m, q.ldq, q.aligned, q.tiles, b.local);
}

template <typename ST>
int thin_q_batched_typed(int32_t count, int32_t maxm, int32_t maxtiles, const ThinQJob *d_jobs,
                         const ThinQBlock *d_map, int64_t nblocks, hipStream_t st) {
  hipLaunchKernelGGL(kq_tu1t, dim3(count, maxm), dim3(256), 0, st, d_jobs);
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL((kq_qhead<ST>), dim3(count, maxm), dim3(256), 0, st, d_jobs);
  RHQR_HIP(hipGetLastError());
  if (nblocks == 0) return RHQR_OK;
  if constexpr (sizeof(ST) >= 4) {
    const unsigned zb = (unsigned)((maxm * QX_NC + 255) / 256);
    hipLaunchKernelGGL(kq_mqt, dim3(count, maxtiles, zb), dim3(256), 0, st, d_jobs);
    RHQR_HIP(hipGetLastError());
    RHQR_LAUNCH(RHQR_PROF_QTAIL, (kq_qtail_mx<ST>), dim3((unsigned)nblocks), dim3(PX_WAVES * 64), 0,
                st, d_jobs, d_map);
  } else {
    hipLaunchKernelGGL((kq_qconv<ST>), dim3(count, maxtiles * QH_NC), dim3(256), 0, st, d_jobs);
    RHQR_HIP(hipGetLastError());
    RHQR_LAUNCH(RHQR_PROF_QTAIL, (kq_qtail16<ST>), dim3((unsigned)nblocks), dim3(QS_WAVES * 64), 0,
                st, d_jobs, d_map);
  }
  return RHQR_OK;
}

// compute units of the current device (cached per device; 256 if unknown)
inline int device_cus() {
  static std::atomic<int> cache[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int c = cache[dev].load(std::memory_order_relaxed);
  if (c > 0) return c;
  if (hipDeviceGetAttribute(&c, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || c < 1)
    c = 256;
  cache[dev].store(c, std::memory_order_relaxed);
  return c;
}

// ------------------------------------------- substitution on matrix cores
// X M = B (m <= 128) with one wave per 16 rows and every unknown of those rows
// kept in registers, so B is read once and X written once.  The columns are
// taken in blocks of 16:
//   X_b = (B_b - sum_{b' < b} X_{b'} M_{b', b}) M_{b, b}^{-1}.
// The products run on v_mfma_f64_16x16x4 (float32 unknowns for float32 and
// 2-byte storage: v_mfma_f32_16x16x4), transposed as in the panel update, so a
// block of unknowns sits in the accumulator layout: lane (g = lane / 16,
// r = lane % 16) holds row r, columns 16 b + di(g, t), t < 4.  That is also
// the layout of a product's right operand once the four columns a step
// consumes are chosen as 16 b' + di(g, t) (one step per earlier block and t):
// the solved blocks enter the products straight from their registers.  The
// 16 x 16 triangle of a block is then solved by forward substitution, every
// lane group redundantly over its row's 16 columns (gathered across the four
// groups), keeping its own four: column c is scaled by 1 / M_cc and removed
// from the later columns at once, so the later columns' sums still add the
// terms k = 0, 1, ... in order.  The coefficients (a padded copy of M, row
// pitch MC + 16 so that the four lane groups' rows fall on different LDS
// banks, identity beyond m, then the reciprocals of the diagonal) are staged
// in LDS once per workgroup; the waves loop over the 16-row strips.
__host__ __device__ inline int trsm_ldp(int mc) { return mc + 16; }
__global__ void k_trsm_pad(int32_t m, int32_t mc, const double *__restrict__ M, int64_t ldm,
                           double *__restrict__ Mp) {
  const int c = blockIdx.x * blockDim.x + threadIdx.x;
  const int k = blockIdx.y;
  const int ldp = trsm_ldp(mc);
  if (c >= ldp) return;
  double v = 0.0;
  if (c < mc) {
    if (k < m && c < m) v = k <= c ? M[k + (int64_t)c * ldm] : 0.0;
    else if (k == c) v = 1.0;
  }
  Mp[(int64_t)k * ldp + c] = v;
  if (k == 0 && c < mc) Mp[(int64_t)mc * ldp + c] = c < m ? 1.0 / M[c + (int64_t)c * ldm] : 1.0;
}

constexpr int TM_WAVES = 16;  // waves per workgroup
template <typename ST, int NB>
__global__ void __launch_bounds__(TM_WAVES * 64) k_trsm_mx(const ST *__restrict__ B, int64_t ldb,
                                                           ST *__restrict__ X, int64_t ldx,
                                                           int64_t rows, int32_t m,
                                                           const double *__restrict__ Mp) {
  using CT = typename CompT<ST>::type;
  using Ops = PxOps<CT>;
  using acc_t = typename Ops::acc_t;
  constexpr int MC = 16 * NB, LDP = MC + 16;
  constexpr int NCOEF = MC * LDP + MC;
  static_assert(NCOEF % 2 == 0, "16-byte staging");
  extern __shared__ double Ml[];
  for (int i = threadIdx.x; i < NCOEF / 2; i += TM_WAVES * 64)
    reinterpret_cast<double2 *>(Ml)[i] = reinterpret_cast<const double2 *>(Mp)[i];
  __syncthreads();
  const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
  const int g = lane >> 4, r = lane & 15;
  const int64_t nstrips = (rows + 15) / 16;
  for (int64_t sidx = (int64_t)blockIdx.x * TM_WAVES + w; sidx < nstrips;
       sidx += (int64_t)gridDim.x * TM_WAVES) {
    const int64_t row = sidx * 16 + r;
    const bool rv = row < rows;
    // the coefficients are the same for every strip and block: an opaque
    // offset keeps their loads next to their use (hoisted, they would take
    // every register)
    int zoff = 0;
    acc_t x[NB];
    // every right-hand side of the strip, loaded at once (clamped indices,
    // so the loads issue together without branches; out-of-range entries
    // are replaced by zeros)
    // column 16 b + di(g, t) = 16 b + di(0, t) + di(g, 0): one per-lane base
    // and uniform offsets (only the last block can reach beyond m)
    const ST *bg = B + (rv ? row : rows - 1) + (int64_t)Ops::di(g, 0) * ldb;
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        if (b + 1 < NB) {
          x[b][t] = cvt_in<CT>(bg[(int64_t)(16 * b + Ops::di(0, t)) * ldb]);
        } else {
          const int col = 16 * b + Ops::di(g, t);
          x[b][t] = cvt_in<CT>(B[(rv ? row : rows - 1) + (int64_t)(col < m ? col : m - 1) * ldb]);
        }
      }
#pragma unroll
    for (int b = 0; b < NB; ++b)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 16 * b + Ops::di(g, t);
        if (!(rv && col < m)) x[b][t] = (CT)0;
      }
#pragma unroll
    for (int b = 0; b < NB; ++b) {
      // this block's coefficient loads stay after the previous block's stores
      asm volatile("" : "+v"(zoff));
      const double *Mq = Ml + zoff;
      // x_b -= X_{b'} M_{b', b}: left operand -M[16 b' + di(g, t)][16 b + r];
      // the next earlier block's operands load while this one's products run
      CT a[4], an[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) a[t] = (CT)(-Mq[Ops::di(g, t) * LDP + 16 * b + r]);
#pragma unroll
      for (int b2 = 0; b2 < b; ++b2) {
        if (b2 + 1 < b) {
#pragma unroll
          for (int t = 0; t < 4; ++t)
            an[t] = (CT)(-Mq[(16 * (b2 + 1) + Ops::di(g, t)) * LDP + 16 * b + r]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) x[b] = Ops::mma(a[t], x[b2][t], x[b]);
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) a[t] = an[t];
      }
      // forward substitution over the diagonal block: column c (held by lane
      // group gc, register tc) is scaled by 1 / M_cc, broadcast to the row's
      // other lane groups and removed from their later columns
      // (each lane scales its own column's value by that column's reciprocal
      // before the broadcast, so no step waits on a load of it)
      const double *md = Mq + 16 * b * LDP + 16 * b;
      const double *iv = Mq + MC * LDP + 16 * b;
      CT cf[4], cn[4], ivr[4];
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        cf[t] = (CT)md[Ops::di(g, t)];
        ivr[t] = (CT)iv[Ops::di(g, t)];
      }
#pragma unroll
      for (int c = 0; c < 16; ++c) {
        int gc = 0, tc = 0;
#pragma unroll
        for (int g2 = 0; g2 < 4; ++g2)
#pragma unroll
          for (int t = 0; t < 4; ++t)
            if (Ops::di(g2, t) == c) {
              gc = g2;
              tc = t;
            }
        if (c + 1 < 16) {
#pragma unroll
          for (int t = 0; t < 4; ++t) cn[t] = (CT)md[(c + 1) * LDP + Ops::di(g, t)];
        }
        __builtin_amdgcn_sched_barrier(0);
        const CT xc = __shfl(x[b][tc] * ivr[tc], 16 * gc + r, 64);
#pragma unroll
        for (int t = 0; t < 4; ++t) {
          const int col = Ops::di(g, t);
          const CT upd = x[b][t] - xc * cf[t];
          x[b][t] = col == c ? xc : (col > c ? upd : x[b][t]);
        }
        __builtin_amdgcn_sched_barrier(0);
#pragma unroll
        for (int t = 0; t < 4; ++t) cf[t] = cn[t];
      }
      ST *xg = X + row + (int64_t)Ops::di(g, 0) * ldx;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int col = 16 * b + Ops::di(g, t);
        if (rv && col < m)
          xg[(int64_t)(16 * b + Ops::di(0, t)) * ldx] = cvt_out<ST>((double)x[b][t]);
      }
    }
  }
}

template <typename ST>
int trsm_blocked_typed(const ST *B, int64_t ldb, int64_t rows, int32_t m, const double *M,
                       int64_t ldm, ST *X, int64_t ldx, double *coef, float *stage,
                       hipStream_t st) {
  if (rows <= 0) return RHQR_OK;
  constexpr int VEC = sizeof(ST) == 8 ? 2 : 4;
  if (sizeof(ST) == 2 && !stage) return RHQR_ERR_WORKSPACE;
  const int aligned = ((uintptr_t)B % 16 == 0) && ((uintptr_t)X % 16 == 0) &&
                      ((ldb * (int64_t)sizeof(ST)) % 16 == 0) &&
                      ((ldx * (int64_t)sizeof(ST)) % 16 == 0) &&
                      (sizeof(ST) != 2 || (uintptr_t)stage % 16 == 0);
  // m <= 128: one pass on matrix cores, every unknown in registers
  if (m <= 128) {
    const int nb16 = (m + 15) / 16, mc = 16 * nb16, ldp = trsm_ldp(mc);
    hipLaunchKernelGGL(k_trsm_pad, dim3((ldp + 255) / 256, mc), dim3(256), 0, st, m, mc, M, ldm,
                       coef);
    RHQR_HIP(hipGetLastError());
    const size_t shm = sizeof(double) * ((size_t)mc * ldp + mc);
    const int64_t strips = (rows + 15) / 16;
    const int64_t wgs = (strips + TM_WAVES - 1) / TM_WAVES;
    // persistent workgroups: as many as the LDS of a compute unit holds (at most two)
    const int64_t per_cu = shm * 2 + 2048 <= 160 * 1024 ? 2 : 1;
    const int64_t cap = per_cu * device_cus();
    const dim3 rg((unsigned)(wgs < cap ? wgs : cap));
#define RHQR_TRSM_MX(NBV)                                                                    \
  case NBV:                                                                                  \
    RHQR_HIP(hipFuncSetAttribute((const void *)k_trsm_mx<ST, NBV>,                           \
                                 hipFuncAttributeMaxDynamicSharedMemorySize, (int)shm));     \
    RHQR_LAUNCH(RHQR_PROF_TRSM, (k_trsm_mx<ST, NBV>), rg, dim3(TM_WAVES * 64), shm, st, B, ldb, \
                X, ldx, rows, m, (const double *)coef);                                      \
    break
    switch (nb16) {
      RHQR_TRSM_MX(1);
      RHQR_TRSM_MX(2);
      RHQR_TRSM_MX(3);
      RHQR_TRSM_MX(4);
      RHQR_TRSM_MX(5);
      RHQR_TRSM_MX(6);
      RHQR_TRSM_MX(7);
      RHQR_TRSM_MX(8);
    }
#undef RHQR_TRSM_MX
    RHQR_HIP(hipGetLastError());
    return RHQR_OK;
  }
  double *Ct = coef, *Md = coef + (size_t)m * TRSM_NB;
  const dim3 grid((unsigned)((rows + (int64_t)PANEL_TPB * VEC - 1) / ((int64_t)PANEL_TPB * VEC)));
  for (int32_t J = 0; J < m; J += TRSM_NB) {
    const int32_t nb = m - J < TRSM_NB ? m - J : TRSM_NB;
    const int kmax = J > TRSM_NB ? J : TRSM_NB;
    hipLaunchKernelGGL(k_trsm_coef, dim3((kmax + 255) / 256, TRSM_NB), dim3(256), 0, st, J, nb, M,
                       ldm, Ct, Md);
    RHQR_HIP(hipGetLastError());
    RHQR_LAUNCH(RHQR_PROF_TRSM, (k_trsm_blk<ST>), grid, dim3(PANEL_TPB), 0, st, B, ldb, X, ldx,
                stage, rows, J, nb, (const double *)Ct, (const double *)Md, aligned);
  }
  return RHQR_OK;
}

}  // namespace

size_t trsm_coef_bytes(int32_t m) {
  // the blocked kernel's tables, or the padded copy of M of the matrix-core kernel
  const size_t blk = (size_t)m * TRSM_NB + 256;
  const size_t mc = 16 * (size_t)((m + 15) / 16);
  const size_t pad = m <= 128 ? mc * (size_t)trsm_ldp((int)mc) + mc : 0;
  return align_up(sizeof(double) * (blk > pad ? blk : pad));
}

size_t trsm_stage_bytes(int dtype, int64_t rows, int32_t m) {
  return dtype_size(dtype) == 2 ? align_up(sizeof(float) * (size_t)((rows + 3) & ~(int64_t)3) * m) : 0;
}

int launch_trsm_blocked(int dtype, const void *B, int64_t ldb, int64_t rows, int32_t m,
                        const double *M, int64_t ldm, void *X, int64_t ldx, double *coef,
                        float *stage, hipStream_t st) {
  switch (dtype) {
    case RHQR_F64:
      return trsm_blocked_typed<double>((const double *)B, ldb, rows, m, M, ldm, (double *)X, ldx,
                                        coef, stage, st);
    case RHQR_F32:
      return trsm_blocked_typed<float>((const float *)B, ldb, rows, m, M, ldm, (float *)X, ldx,
                                       coef, stage, st);
    case RHQR_F16:
      return trsm_blocked_typed<__half>((const __half *)B, ldb, rows, m, M, ldm, (__half *)X, ldx,
                                        coef, stage, st);
    case RHQR_BF16:
      return trsm_blocked_typed<__hip_bfloat16>((const __hip_bfloat16 *)B, ldb, rows, m, M, ldm,
                                                (__hip_bfloat16 *)X, ldx, coef, stage, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

ColProblem make_col_problem(const LoopArgs &a, const LoopWs &w, int tpw) {
  ColProblem P;
  const size_t es = dtype_size(a.dtype);
  P.W = a.W;
  P.ldw = a.ldw;
  P.n = a.n;
  P.m = a.m;
  P.l = a.l;
  P.Z = a.Z;
  P.ldz = a.ldz;
  P.S = a.S;
  P.lds = a.lds;
  P.T = a.T;
  P.ldt = a.ldt;
  P.R = a.R;
  P.ldr = a.ldr;
  P.signs = a.signs;
  P.rows = a.rows;
  P.omega = a.omega;
  P.scale = a.kind == RHQR_SKETCH_SRHT ? 1.0 / std::sqrt((double)a.l) : 1.0;
  P.nparts = (a.n + (int64_t)TILE * tpw - 1) / ((int64_t)TILE * tpw);
  P.gred = (a.m + RED_CHUNK - 1) / RED_CHUNK + (a.l + RED_CHUNK - 1) / RED_CHUNK;
  P.scaling = a.scaling;
  P.defer = a.defer;
  P.c0 = a.c0;
  P.aligned = ((uintptr_t)a.W % 16 == 0) && ((a.ldw * (int64_t)es) % 16 == 0);
  P.part = w.part;
  P.y = w.y;
  P.sq = w.sq;
  P.dpart = w.dpart;
  P.epart = w.epart;
  P.ypart = w.ypart;
  P.scal = w.scal;
  P.c = w.c;
  P.cf = w.cf;
  P.ia = w.ia;
  P.Tt = w.Tt;
  P.dcpart = w.dcpart;
  P.fs = w.fs;
  P.status = w.status;
  P.C = P.G = nullptr;
  return P;
}

int launch_fill(void *p, size_t bytes, hipStream_t st) {
  const size_t nw = bytes / 4;
  if (nw == 0) return RHQR_OK;
  hipLaunchKernelGGL(k_fill, dim3((nw + 255) / 256), dim3(256), 0, st, (uint32_t *)p, nw);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

size_t loop_ws_bytes(int kind, int dtype, int64_t n, int32_t m, int32_t l) {
  const int32_t L = l + m;
  const int64_t ntiles = (n + TILE - 1) / TILE;
  const int gred = (m + RED_CHUNK - 1) / RED_CHUNK + (l + RED_CHUNK - 1) / RED_CHUNK;
  const int gss = (L + RED_CHUNK - 1) / RED_CHUNK;
  size_t b = 0;
  b += align_up(sizeof(int32_t) * 4);
  b += align_up(sizeof(double) * (MAXM / FIN_P));
  b += align_up(sizeof(double) * 4);
  b += align_up(sizeof(double) * L);
  b += align_up(sizeof(double) * gred);
  b += 2 * align_up(sizeof(double) * (size_t)gred * m);
  b += align_up(sizeof(double) * gred);
  b += align_up(sizeof(double) * 4 * m);
  b += 3 * align_up(sizeof(double) * m);
  b += align_up(sizeof(double) * (size_t)m * m);
  if (kind != RHQR_SKETCH_IDENT) b += align_up(sizeof(double) * (size_t)ntiles * l);
  return b;
}

int loop_ws_carve(void *ws, size_t bytes, int kind, int dtype, int64_t n, int32_t m, int32_t l,
                  LoopWs *o) {
  if (bytes < loop_ws_bytes(kind, dtype, n, m, l)) return RHQR_ERR_WORKSPACE;
  const int32_t L = l + m;
  const int64_t ntiles = (n + TILE - 1) / TILE;
  const int gred = (m + RED_CHUNK - 1) / RED_CHUNK + (l + RED_CHUNK - 1) / RED_CHUNK;
  const int gss = (L + RED_CHUNK - 1) / RED_CHUNK;
  char *p = (char *)ws;
  auto take = [&](size_t b) {
    char *r = p;
    p += align_up(b);
    return (void *)r;
  };
  o->status = (int32_t *)take(sizeof(int32_t) * 4);
  o->dcpart = (double *)take(sizeof(double) * (MAXM / FIN_P));
  o->fs = (double *)take(sizeof(double) * 4);
  o->y = (double *)take(sizeof(double) * L);
  o->sq = (double *)take(sizeof(double) * gred);
  o->dpart = (double *)take(sizeof(double) * (size_t)gred * m);
  o->epart = (double *)take(sizeof(double) * (size_t)gred * m);
  o->ypart = (double *)take(sizeof(double) * gred);
  o->scal = (double *)take(sizeof(double) * 4 * m);
  o->c = (double *)take(sizeof(double) * m);
  o->cf = (double *)take(sizeof(double) * m);
  o->ia = (double *)take(sizeof(double) * m);
  o->Tt = (double *)take(sizeof(double) * (size_t)m * m);
  o->part = kind != RHQR_SKETCH_IDENT ? (double *)take(sizeof(double) * (size_t)ntiles * l) : nullptr;
  o->skws = nullptr;
  o->skws_bytes = 0;
  return RHQR_OK;
}

#define RHQR_DISPATCH(dt, expr)                                        \
  switch (dt) {                                                        \
    case RHQR_F64: { using ST = double; return expr; }                 \
    case RHQR_F32: { using ST = float; return expr; }                  \
    case RHQR_F16: { using ST = __half; return expr; }                 \
    case RHQR_BF16: { using ST = __hip_bfloat16; return expr; }        \
  }                                                                    \
  return RHQR_ERR_UNSUPPORTED;

int engine_tall(const LoopArgs &a, const LoopWs &w, int32_t j, hipStream_t st) {
  RHQR_DISPATCH(a.dtype, tall_typed<ST>(a, w, j, 0, st))
}


int run_column_loop_blocked(const LoopArgs &a, const LoopWs &w, int panel, int outer, double *C,
                            double *G, hipStream_t st) {
  if (a.m > MAXM) return RHQR_ERR_UNSUPPORTED;
  RHQR_DISPATCH(a.dtype, run_blocked_typed<ST>(a, w, panel, outer, C, G, st))
}

int run_column_loop_alg5(const rhqr_sketch_s *h, const LoopArgs &a, const LoopWs &w, int b,
                         double *C, double *G, double *Z, void *skws, size_t skws_bytes,
                         hipStream_t st) {
  if (a.m > MAXM) return RHQR_ERR_UNSUPPORTED;
  RHQR_DISPATCH(a.dtype, run_alg5_typed<ST>(h, a, w, b, C, G, Z, skws, skws_bytes, st))
}

int engine_step(const LoopArgs &a, const LoopWs &w, int32_t j, int next, hipStream_t st) {
  if (a.m > MAXM) return RHQR_ERR_UNSUPPORTED;
  RHQR_DISPATCH(a.dtype, step_typed<ST>(a, w, j, next, st))
}

int run_column_loop(const LoopArgs &a, const LoopWs &w, hipStream_t st) {
  if (a.m > MAXM) return RHQR_ERR_UNSUPPORTED;
  switch (a.dtype) {
    case RHQR_F64: return run_typed<double>(a, w, st);
    case RHQR_F32: return run_typed<float>(a, w, st);
    case RHQR_F16: return run_typed<__half>(a, w, st);
    case RHQR_BF16: return run_typed<__hip_bfloat16>(a, w, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

int64_t thin_q_tail_blocks(int dtype, int64_t n, int32_t m, int32_t *tiles, int64_t *groups,
                           int32_t *Kp) {
  const int es = (int)dtype_size(dtype);
  const int64_t rows = n - m;
  *Kp = (m + PM_KP - 1) / PM_KP * PM_KP;
  if (es >= 4) {
    *tiles = (m + QX_NC - 1) / QX_NC;
    *groups = panel_mx_groups(n, m, es);
  } else {
    *tiles = (m + QH_NC - 1) / QH_NC;
    const int64_t waves = (rows + PM_ROWS - 1) / PM_ROWS;
    *groups = (waves + QS_WAVES - 1) / QS_WAVES;
  }
  if (rows <= 0) return 0;
  return (*groups + 7) / 8 * 8 * *tiles;
}

int launch_thin_q_batched(int dtype, int32_t count, int32_t maxm, int32_t maxtiles,
                          const ThinQJob *d_jobs, const ThinQBlock *d_map, int64_t nblocks,
                          hipStream_t st) {
  if (count < 1 || maxm < 1) return RHQR_OK;
  switch (dtype) {
    case RHQR_F64:
      return thin_q_batched_typed<double>(count, maxm, maxtiles, d_jobs, d_map, nblocks, st);
    case RHQR_F32:
      return thin_q_batched_typed<float>(count, maxm, maxtiles, d_jobs, d_map, nblocks, st);
    case RHQR_F16:
      return thin_q_batched_typed<__half>(count, maxm, maxtiles, d_jobs, d_map, nblocks, st);
    case RHQR_BF16:
      return thin_q_batched_typed<__hip_bfloat16>(count, maxm, maxtiles, d_jobs, d_map, nblocks,
                                                  st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

size_t thin_q_bytes(int32_t m) {
  // the larger of: split coefficients (2-byte storage, unaligned columns) and
  // Mq in the tile layout of the matrix-core product
  const size_t Kp = (size_t)(m + PM_KP - 1) / PM_KP * PM_KP;
  const size_t tiles = (size_t)(m + QH_NC - 1) / QH_NC;
  const size_t split = 2 * tiles * Kp * QH_NC * sizeof(unsigned short) + tiles * QH_NC * sizeof(float);
  const size_t xt = (size_t)(m + QX_NC - 1) / QX_NC * QX_NC * (size_t)m * sizeof(double);
  return align_up(split > xt ? split : xt);
}

int launch_thin_q(int dtype, int64_t n, int32_t m, const void *U, int64_t ldu, const double *S,
                  int64_t lds, const double *T, int64_t ldt, double *Mq, void *qmf, void *Q,
                  int64_t ldq, hipStream_t st) {
  switch (dtype) {
    case RHQR_F64:
      return thin_q_typed<double>(n, m, (const double *)U, ldu, S, lds, T, ldt, Mq, qmf,
                                  (double *)Q, ldq, st);
    case RHQR_F32:
      return thin_q_typed<float>(n, m, (const float *)U, ldu, S, lds, T, ldt, Mq, qmf, (float *)Q,
                                 ldq, st);
    case RHQR_F16:
      return thin_q_typed<__half>(n, m, (const __half *)U, ldu, S, lds, T, ldt, Mq, qmf,
                                  (__half *)Q, ldq, st);
    case RHQR_BF16:
      return thin_q_typed<__hip_bfloat16>(n, m, (const __hip_bfloat16 *)U, ldu, S, lds, T, ldt, Mq,
                                          qmf, (__hip_bfloat16 *)Q, ldq, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}
