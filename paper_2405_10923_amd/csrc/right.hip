// Right-looking RHQR (Alg. 3) on the GPU, selected by bit 29 of rhqr_factor's
// options.  Step j (0-based) of the column loop:
//   1. [y Y] = Psi W_{:, j:m}: the m - j trailing columns sketched afresh by
//      the multi-column sketch (Alg. 1), one synchronisation per step;
//   2. RHVector (Alg. 2) of w_j from y, in one workgroup: s_j -> S_{:, j},
//      R_{:, j}; then, one wave per product over several workgroups, the
//      coefficients c_k = beta_j s_j^t Y_{:, k} of the trailing columns and
//      a = S^t s_j.  T_{:, j} = -beta_j T a follows the recursion of Alg. 4,
//      so the outputs are those of the left-looking forms (formed by one
//      extra workgroup of step 3's launch);
//   3. one pass over the n rows: u_j = w_j / alpha_j (the head rows are s_j's:
//      the head block of Psi is the identity), stored over w_j, and
//      W_{:, k} -= u_j c_k for every trailing column k.
// Per step the pass reads and writes the m - j - 1 trailing columns and the
// sketch reads the m - j columns again: about 3 n m^2 / 2 elements over the
// factorization against n m^2 / 2 for the refresh passes of Alg. 4 (Alg. 3
// sketches m - j + 1 vectors at step j, which is why the left-looking form is
// the one the paper runs at scale).
#include "colstep.h"

#include "engine.h"

namespace {

constexpr int R3_TPB = 1024;  // workgroups of step 2 (RHVector; products, 16 per workgroup)
constexpr int AP_TPB = 256;   // the row pass of step 3
constexpr int AP_RPT = 4;     // rows per thread (strided by AP_TPB)

// Step 2 of column j, RHVector.  Zr: the (l+m) x (m-j) sketch [y Y] (ld ldz).
// Writes S_{:, j}, R_{:, j}, T_{j, j} = beta_j (T is zero below), ia[j] =
// 1/alpha_j (0 for an identity reflector) and the breakdown / non-finite
// flags of column j.
__global__ void __launch_bounds__(R3_TPB) k_r3_vec(int32_t L, int32_t m, int32_t j,
                                                   const double *__restrict__ Zr, int scaling,
                                                   double *__restrict__ S, int64_t lds,
                                                   double *__restrict__ T, int64_t ldt,
                                                   double *__restrict__ R, int64_t ldr,
                                                   double *__restrict__ ia,
                                                   int32_t *__restrict__ status) {
  __shared__ double red[R3_TPB / 64];
  __shared__ StepScalars shs;
  const int tid = threadIdx.x;
  // rho^2 over the rows k >= j of y (every thread its strided rows, then the
  // workgroup sum: fixed order)
  double ss = 0.0;
  for (int k = j + tid; k < L; k += R3_TPB) ss += Zr[k] * Zr[k];
  ss = block_sum(ss, red);
  if (tid == 0) shs = step_scalars(Zr[j], ss, scaling);
  __syncthreads();
  const StepScalars sc = shs;
  // s_j = ((0; y_{j:}) + sigma rho e_j) / alpha (e_j for an identity reflector;
  // the pivot entry is exactly 1 in the unit-pivot scaling)
  for (int k = tid; k < L; k += R3_TPB) {
    double v = 0.0;
    if (k == j)
      v = sc.ident ? 1.0 : (scaling == RHQR_SCALE_UNIT_PIVOT ? 1.0 : sc.gamma / sc.alpha);
    else if (k > j)
      v = sc.ident ? 0.0 : Zr[k] / sc.alpha;
    S[k + (int64_t)j * lds] = v;
  }
  for (int r = tid; r < m; r += R3_TPB)
    R[r + (int64_t)j * ldr] = r < j ? Zr[r] : (r == j ? -sc.sigma * sc.rho : 0.0);
  if (tid == 0) {
    T[j + (int64_t)j * ldt] = sc.beta;
    ia[j] = sc.ident ? 0.0 : 1.0 / sc.alpha;
    if (sc.ident) atomicCAS(status, 0, j + 1);
    if (sc.nonfinite) atomicCAS(status + 1, 0, j + 1);
  }
}

// Step 2 of column j, products: wave w of workgroup b takes p = 16 b + w
// (p < m - 1).  p < j: a_p = S_{:, p}^t s_j; p >= j: trailing column k = p + 1,
// coef[k] = beta_j (Psi w_k)^t s_j with Psi w_k = Zr_{:, k - j}.  Lanes over
// the rows k >= j (s_j is zero above its pivot), one wave_sum per product:
// fixed order.  beta_j is read from T_{j, j}.
__global__ void __launch_bounds__(R3_TPB) k_r3_dots(int32_t L, int32_t m, int32_t j,
                                                    const double *__restrict__ Zr, int64_t ldz,
                                                    const double *__restrict__ S, int64_t lds,
                                                    const double *__restrict__ T, int64_t ldt,
                                                    double *__restrict__ a,
                                                    double *__restrict__ coef) {
  extern __shared__ double s[];  // s_j (rows >= j), L entries
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const double *__restrict__ sj = S + (int64_t)j * lds;
  for (int k = j + tid; k < L; k += R3_TPB) s[k] = sj[k];
  const double beta = T[j + (int64_t)j * ldt];
  __syncthreads();
  const int p = blockIdx.x * (R3_TPB / 64) + w;
  if (p >= m - 1) return;  // the whole wave (no barrier follows)
  const double *__restrict__ col = p < j ? S + (int64_t)p * lds : Zr + (int64_t)(p + 1 - j) * ldz;
  double acc = 0.0;
#pragma unroll 4
  for (int k = j + lane; k < L; k += 64) acc += col[k] * s[k];
  acc = wave_sum(acc);
  if (lane == 0) {
    if (p < j)
      a[p] = acc;
    else
      coef[p + 1] = beta * acc;
  }
}

// Step 3 of column j: thread t of workgroup b owns the rows
// b AP_TPB AP_RPT + t + AP_TPB i.  u_r = S_{r, j} for r < m, w_{r, j} / alpha_j
// otherwise, rounded to the storage type and stored over w_j; the trailing
// columns are updated with the stored value (so the stored U reproduces the
// update), in the computation type.
// The last workgroup of the launch forms T_{p, j} = -beta_j sum_{q = p}^{j-1}
// T_{p, q} a_q instead (one wave per p, lanes over q, one wave_sum each).
template <typename ST>
__global__ void __launch_bounds__(AP_TPB) k_r3_apply(ST *__restrict__ W, int64_t ldw, int64_t n,
                                                     int32_t m, int32_t j,
                                                     const double *__restrict__ S, int64_t lds,
                                                     const double *__restrict__ ia,
                                                     const double *__restrict__ coef,
                                                     double *__restrict__ T, int64_t ldt,
                                                     const double *__restrict__ a) {
  using CT = typename CompT<ST>::type;
  if (blockIdx.x == gridDim.x - 1) {
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const double beta = T[j + (int64_t)j * ldt];
    for (int p = w; p < j; p += AP_TPB / 64) {
      double t = 0.0;
      for (int q = p + lane; q < j; q += 64) t += T[p + (int64_t)q * ldt] * a[q];
      t = wave_sum(t);
      if (lane == 0) T[p + (int64_t)j * ldt] = -beta * t;
    }
    return;
  }
  const int64_t base = (int64_t)blockIdx.x * (AP_TPB * AP_RPT) + threadIdx.x;
  const double iaj = ia[j];
  ST *__restrict__ wj = W + (int64_t)j * ldw;
  CT u[AP_RPT];
#pragma unroll
  for (int i = 0; i < AP_RPT; ++i) {
    const int64_t r = base + (int64_t)AP_TPB * i;
    u[i] = 0;
    if (r < n) {
      const double v = r < m ? S[r + (int64_t)j * lds] : (double)cvt_in<CT>(wj[r]) * iaj;
      const ST q = cvt_out<ST>(v);
      wj[r] = q;
      u[i] = cvt_in<CT>(q);
    }
  }
#pragma unroll 2
  for (int32_t k = j + 1; k < m; ++k) {
    const CT ck = (CT)coef[k];
    ST *__restrict__ wk = W + (int64_t)k * ldw;
    CT x[AP_RPT];
#pragma unroll
    for (int i = 0; i < AP_RPT; ++i) {
      const int64_t r = base + (int64_t)AP_TPB * i;
      x[i] = r < n ? cvt_in<CT>(wk[r]) : (CT)0;
    }
#pragma unroll
    for (int i = 0; i < AP_RPT; ++i) {
      const int64_t r = base + (int64_t)AP_TPB * i;
      if (r < n) wk[r] = cvt_out<ST>((double)(x[i] - u[i] * ck));
    }
  }
}

template <typename ST>
int launch_apply(const LoopArgs &a, const LoopWs &w, int32_t j, hipStream_t st) {
  const int64_t rows_per_wg = (int64_t)AP_TPB * AP_RPT;
  const int64_t nwg = (a.n + rows_per_wg - 1) / rows_per_wg;
  RHQR_LAUNCH(RHQR_PROF_RIGHT_APPLY, k_r3_apply<ST>, dim3((unsigned)(nwg + 1)), dim3(AP_TPB), 0,
              st, (ST *)a.W, a.ldw, a.n, a.m, j, (const double *)a.S, a.lds, (const double *)w.ia,
              (const double *)w.c, a.T, a.ldt, (const double *)w.cf);
  return RHQR_OK;
}

}  // namespace

int run_column_loop_right(const rhqr_sketch_s *h, const LoopArgs &a, const LoopWs &w, double *Z,
                          void *skws, size_t skws_bytes, hipStream_t st) {
  const int32_t m = a.m, L = a.l + a.m;
  if (m > MAXM) return RHQR_ERR_UNSUPPORTED;
  const size_t es = dtype_size(a.dtype);
  const size_t shm = sizeof(double) * (size_t)L;
  if (shm > 64 * 1024) return RHQR_ERR_UNSUPPORTED;
  RHQR_HIP(hipFuncSetAttribute((const void *)k_r3_dots, hipFuncAttributeMaxDynamicSharedMemorySize,
                               (int)shm));
  for (int32_t j = 0; j < m; ++j) {
    const void *Wj = (const char *)a.W + (size_t)j * (size_t)a.ldw * es;
    int rc = launch_sketch(h, a.dtype, a.n, m - j, Wj, a.ldw, Z, L, skws, skws_bytes, st);
    if (rc) return rc;
    RHQR_LAUNCH(RHQR_PROF_RIGHT_VEC, k_r3_vec, dim3(1), dim3(R3_TPB), 0, st, L, m, j,
                (const double *)Z, a.scaling, a.S, a.lds, a.T, a.ldt, a.R, a.ldr, w.ia, w.status);
    if (m > 1)
      RHQR_LAUNCH(RHQR_PROF_RIGHT_VEC, k_r3_dots, dim3((m - 1 + R3_TPB / 64 - 1) / (R3_TPB / 64)),
                  dim3(R3_TPB), shm, st, L, m, j, (const double *)Z, (int64_t)L,
                  (const double *)a.S, a.lds, (const double *)a.T, a.ldt, w.cf, w.c);
    switch (a.dtype) {
      case RHQR_F64: rc = launch_apply<double>(a, w, j, st); break;
      case RHQR_F32: rc = launch_apply<float>(a, w, j, st); break;
      case RHQR_F16: rc = launch_apply<__half>(a, w, j, st); break;
      default: rc = launch_apply<__hip_bfloat16>(a, w, j, st);
    }
    if (rc) return rc;
  }
  return RHQR_OK;
}
