// C ABI: rhqr_factor (left-looking RHQR, Alg. 4), its allocation-free variant
// rhqr_factor_noalloc, BLAS2-RGS (Alg. 9) and rhqr_status.
#include "engine.h"

#include <mutex>
#include <vector>

namespace {

__global__ void k_zero_sq(double *A, int64_t lda, int32_t rows, int32_t cols) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r < rows && c < cols) A[r + (int64_t)c * lda] = 0.0;
}

struct FactorWs {
  LoopWs loop;
  double *Z;
  void *skws;
  size_t skws_bytes;
  double *Mq;
  double *C, *G;  // panel coefficients (blocked schedule), m x 32 each
  void *qmf;      // split coefficients of the matrix-core thin Q
};

// the multi-column sketch workspace for any number of columns up to m (the
// pre-sketch takes m, block RHQR one block of at most 32, right-looking RHQR
// the m - j trailing columns; fewer columns can take more partial groups each)
size_t factor_sketch_ws(const rhqr_sketch_s *h, int32_t m) {
  size_t b = 0;
  for (int32_t k = 1; k <= m; ++k) {
    const size_t bk = sketch_ws_bytes(h, k);
    if (bk > b) b = bk;
  }
  return b;
}

size_t factor_ws_bytes(const rhqr_sketch_s *h, int dtype, int32_t m) {
  const int32_t L = h->l + m;
  size_t b = loop_ws_bytes(h->kind, dtype, h->n, m, h->l);
  b += align_up(sizeof(double) * (size_t)L * m);
  b += align_up(factor_sketch_ws(h, m));
  b += align_up(sizeof(double) * (size_t)m * m);
  b += 2 * align_up(sizeof(double) * (size_t)m * 32);
  b += thin_q_bytes(m);
  return b;
}

int factor_ws_carve(const rhqr_sketch_s *h, int dtype, int32_t m, void *ws, size_t bytes,
                    FactorWs *o) {
  if (bytes < factor_ws_bytes(h, dtype, m)) return RHQR_ERR_WORKSPACE;
  const size_t lb = loop_ws_bytes(h->kind, dtype, h->n, m, h->l);
  int rc = loop_ws_carve(ws, lb, h->kind, dtype, h->n, m, h->l, &o->loop);
  if (rc) return rc;
  char *p = (char *)ws + lb;
  const int32_t L = h->l + m;
  o->Z = (double *)p;
  p += align_up(sizeof(double) * (size_t)L * m);
  o->skws = p;
  o->skws_bytes = align_up(factor_sketch_ws(h, m));
  p += o->skws_bytes;
  o->Mq = (double *)p;
  p += align_up(sizeof(double) * (size_t)m * m);
  o->C = (double *)p;
  p += align_up(sizeof(double) * (size_t)m * 32);
  o->G = (double *)p;
  p += align_up(sizeof(double) * (size_t)m * 32);
  o->qmf = p;
  return RHQR_OK;
}

}  // namespace

extern "C" size_t rhqr_factor_workspace_size(rhqr_sketch_t h, int dtype, int32_t m) {
  if (!h || m < 1 || m != h->m || dtype < RHQR_F64 || dtype > RHQR_BF16) return 0;
  return factor_ws_bytes(h, dtype, m);
}

namespace {

bool opts_ok(int opts) {
  const int scaling = opts & 0xff;
  const int panel = (opts >> 8) & 0xff;
  const int outer = (opts >> 16) & 0xff;
  const int tpw = (opts >> 24) & 0xf;
  const bool alg5 = (opts >> 28) & 1;
  const bool alg3 = (opts >> 29) & 1;
  return !((scaling != RHQR_SCALE_UNIT_PIVOT && scaling != RHQR_SCALE_SQRT2) || panel > 32 ||
           ((unsigned)opts >> 30) != 0 ||
           (alg3 && (opts & 0x1fffff00) != 0) || (tpw != 0 && tpw != 1 && tpw != 2 && tpw != 4) ||
           (alg5 && (panel < 1 || outer != 0)) ||
           (outer != 0 && (panel < 2 || outer <= panel || outer > 32 || outer % panel != 0)));
}

// the factorization itself, arguments validated and the workspace carved
int factor_core(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W, int64_t ldw,
                double *d_S, int64_t lds, double *d_T, int64_t ldt, double *d_R, int64_t ldr,
                void *d_Q, int64_t ldq, int opts, const FactorWs &w, hipStream_t st) {
  const int scaling = opts & 0xff;
  const int panel = (opts >> 8) & 0xff;
  const int outer = (opts >> 16) & 0xff;
  const int32_t L = h->l + m;
  int rc;

  rc = launch_fill(w.loop.status, 16, st);
  if (rc) return rc;
  hipLaunchKernelGGL(k_zero_sq, dim3((m + 255) / 256, m), dim3(256), 0, st, d_T, ldt, m, m);
  RHQR_HIP(hipGetLastError());
  const bool alg5 = (opts >> 28) & 1;
  const bool alg3 = (opts >> 29) & 1;

  // pre-sketch of every column: "if next vector available, sketch it now"
  // (block RHQR sketches each block afresh instead, right-looking RHQR the
  // trailing columns at every step)
  if (!alg5 && !alg3) {
    rc = launch_sketch(h, dtype, n, m, d_W, ldw, w.Z, L, w.skws, w.skws_bytes, st);
    if (rc) return rc;
  }

  LoopArgs a;
  a.kind = h->kind;
  a.dtype = dtype;
  a.n = n;
  a.m = m;
  a.l = h->l;
  a.W = d_W;
  a.ldw = ldw;
  a.Z = w.Z;
  a.ldz = L;
  a.S = d_S;
  a.lds = lds;
  a.T = d_T;
  a.ldt = ldt;
  a.R = d_R;
  a.ldr = ldr;
  a.scaling = scaling;
  a.signs = h->d_signs;
  a.rows = h->d_rows;
  a.omega = h->d_omega;
  a.defer = 1;
  a.tpw = (opts >> 24) & 0xf;
  if (alg3)
    rc = run_column_loop_right(h, a, w.loop, w.Z, w.skws, w.skws_bytes, st);
  else if (alg5)
    rc = run_column_loop_alg5(h, a, w.loop, panel, w.C, w.G, w.Z, w.skws, w.skws_bytes, st);
  else
    rc = panel >= 2 ? run_column_loop_blocked(a, w.loop, panel, outer, w.C, w.G, st)
                    : run_column_loop(a, w.loop, st);
  if (rc) return rc;
  if (d_Q) rc = launch_thin_q(dtype, n, m, d_W, ldw, d_S, lds, d_T, ldt, w.Mq, w.qmf, d_Q, ldq, st);
  return rc;
}

__global__ void k_neg_sq(double *A, int64_t lda, int32_t m) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r < m) A[r + (int64_t)c * lda] = -A[r + (int64_t)c * lda];
}

template <typename ST>
__global__ void k_zero_head(ST *A, int64_t lda, int32_t m) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  const int c = blockIdx.y;
  if (r < m) A[r + (int64_t)c * lda] = cvt_out<ST>(0.0);
}

// rows m .. m+n-1 of Qw <- W (n x m), rows 0 .. m-1 <- 0, in the storage type
template <typename ST>
int stage_zero_topped(const void *W, int64_t ldw, int64_t n, int32_t m, void *Qw, int64_t ldq,
                      hipStream_t st) {
  const size_t es = sizeof(ST);
  RHQR_HIP(hipMemcpy2DAsync((char *)Qw + (size_t)m * es, (size_t)ldq * es, W, (size_t)ldw * es,
                            (size_t)n * es, (size_t)m, hipMemcpyDeviceToDevice, st));
  hipLaunchKernelGGL((k_zero_head<ST>), dim3((m + 255) / 256, m), dim3(256), 0, st, (ST *)Qw,
                     ldq, m);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

}  // namespace

extern "C" int rhqr_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W,
                           int64_t ldw, double *d_S, int64_t lds, double *d_T, int64_t ldt,
                           double *d_R, int64_t ldr, void *d_Q, int64_t ldq, int opts,
                           void *d_ws, size_t ws_bytes, void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (m < 1 || m != h->m) return -4;
  if (!d_W) return -5;
  if (ldw < n) return -6;
  const int32_t L = h->l + m;
  if (!d_S) return -7;
  if (lds < L) return -8;
  if (!d_T) return -9;
  if (ldt < m) return -10;
  if (!d_R) return -11;
  if (ldr < m) return -12;
  if (d_Q && ldq < n) return -14;
  if (!opts_ok(opts)) return -15;
  if (!d_ws) return -16;
  if (m > 1024) return RHQR_ERR_UNSUPPORTED;
  FactorWs w;
  const int rc = factor_ws_carve(h, dtype, m, d_ws, ws_bytes, &w);
  if (rc) return rc;
  return factor_core(h, dtype, n, m, d_W, ldw, d_S, lds, d_T, ldt, d_R, ldr, d_Q, ldq, opts, w,
                     (hipStream_t)stream);
}

extern "C" size_t rhqr_rgs_workspace_size(rhqr_sketch_t h, int dtype, int32_t m) {
  return rhqr_factor_workspace_size(h, dtype, m);
}

extern "C" int rhqr_rgs_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, const void *d_W,
                               int64_t ldw, void *d_Q, int64_t ldq, double *d_S, int64_t lds,
                               double *d_T, int64_t ldt, double *d_R, int64_t ldr, int opts,
                               void *d_ws, size_t ws_bytes, void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n < 1 || n + m != h->n) return -3;
  if (m < 1 || m != h->m) return -4;
  if (!d_W) return -5;
  if (ldw < n) return -6;
  if (!d_Q) return -7;
  if (ldq < n + m) return -8;
  const int32_t L = h->l + m;
  if (!d_S) return -9;
  if (lds < L) return -10;
  if (!d_T) return -11;
  if (ldt < m) return -12;
  if (!d_R) return -13;
  if (ldr < m) return -14;
  if (!opts_ok(opts) || (opts & 0xff) != RHQR_SCALE_UNIT_PIVOT) return -15;
  if (!d_ws) return -16;
  if (m > 1024) return RHQR_ERR_UNSUPPORTED;
  FactorWs w;
  int rc = factor_ws_carve(h, dtype, m, d_ws, ws_bytes, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  switch (dtype) {
    case RHQR_F64: rc = stage_zero_topped<double>(d_W, ldw, n, m, d_Q, ldq, st); break;
    case RHQR_F32: rc = stage_zero_topped<float>(d_W, ldw, n, m, d_Q, ldq, st); break;
    case RHQR_F16: rc = stage_zero_topped<__half>(d_W, ldw, n, m, d_Q, ldq, st); break;
    default: rc = stage_zero_topped<__hip_bfloat16>(d_W, ldw, n, m, d_Q, ldq, st);
  }
  if (rc) return rc;
  // left-looking RHQR of [0; W]: the head of every refreshed column below its
  // pivot is exactly zero, so sigma = +1, alpha = rho and beta = 1 throughout
  rc = factor_core(h, dtype, n + m, m, d_Q, ldq, d_S, lds, d_T, ldt, d_R, ldr, nullptr, 0, opts,
                   w, st);
  if (rc) return rc;
  // U = [I; Q] with R_RHQR = -R: Alg. 9's R has the positive diagonal rho_j
  hipLaunchKernelGGL(k_neg_sq, dim3((m + 255) / 256, m), dim3(256), 0, st, d_R, ldr, m);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

extern "C" int rhqr_status(const void *d_ws, void *stream, int32_t *h_info) {
  if (!d_ws) return -1;
  if (!h_info) return -3;
  hipStream_t st = (hipStream_t)stream;
  int32_t w[2] = {0, 0};  // first breakdown, first non-finite column (1-based)
  RHQR_HIP(hipMemcpyAsync(w, d_ws, sizeof(w), hipMemcpyDeviceToHost, st));
  RHQR_HIP(hipStreamSynchronize(st));
  *h_info = w[1] ? -w[1] : w[0];
  return RHQR_OK;
}

// ------------------------------------------------- allocation-free variant
// The workspace of rhqr_factor_noalloc lives in a file-scope device array:
// every GPU the library runs on holds its own copy for the life of the
// process.  In host code `scratch` names a host-side stand-in, not device
// memory: its device address is looked up once per device with
// hipGetSymbolAddress and only that address is ever passed to kernels.
static __device__ __align__(256) unsigned char scratch[RHQR_NOALLOC_SCRATCH_BYTES];

namespace {

// d_info[0] = first breakdown column, d_info[1] = first non-finite column
__global__ void k_copy_status(const int32_t *status, int32_t *info) {
  if (threadIdx.x < 2) info[threadIdx.x] = status[threadIdx.x];
}

struct ScratchTable {
  std::mutex mu;
  std::vector<void *> ptr;  // device address of `scratch`, per device ordinal
};

ScratchTable &scratch_table() {
  static ScratchTable t;
  return t;
}

// device address of this device's copy of `scratch` (the current device)
int scratch_address(void **out) {
  int dev = 0;
  RHQR_HIP(hipGetDevice(&dev));
  ScratchTable &t = scratch_table();
  std::lock_guard<std::mutex> lk(t.mu);
  if ((int)t.ptr.size() <= dev) t.ptr.resize(dev + 1, nullptr);
  if (!t.ptr[dev]) {
    void *p = nullptr;
    RHQR_HIP(hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)));
    if (!p) return RHQR_ERR_HIP;
    t.ptr[dev] = p;
  }
  *out = t.ptr[dev];
  return RHQR_OK;
}

}  // namespace

extern "C" int rhqr_factor_noalloc(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W,
                                   int64_t ldw, double *d_S, int64_t lds, double *d_T,
                                   int64_t ldt, double *d_R, int64_t ldr, void *d_Q, int64_t ldq,
                                   int opts, int32_t *d_info, void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (m < 1 || m != h->m) return -4;
  if (!d_W) return -5;
  if (ldw < n) return -6;
  const int32_t L = h->l + m;
  if (!d_S) return -7;
  if (lds < L) return -8;
  if (!d_T) return -9;
  if (ldt < m) return -10;
  if (!d_R) return -11;
  if (ldr < m) return -12;
  if (d_Q && ldq < n) return -14;
  if (!opts_ok(opts)) return -15;
  if (m > 1024) return RHQR_ERR_UNSUPPORTED;
  const size_t need = factor_ws_bytes(h, dtype, m);
  if (need > RHQR_NOALLOC_SCRATCH_BYTES) return RHQR_ERR_WORKSPACE;
  void *ws = nullptr;
  int rc = scratch_address(&ws);
  if (rc) return rc;
  FactorWs w;
  rc = factor_ws_carve(h, dtype, m, ws, need, &w);
  if (rc) return rc;
  hipStream_t st = (hipStream_t)stream;
  rc = factor_core(h, dtype, n, m, d_W, ldw, d_S, lds, d_T, ldt, d_R, ldr, d_Q, ldq, opts, w, st);
  if (rc || !d_info) return rc;
  hipLaunchKernelGGL(k_copy_status, dim3(1), dim3(64), 0, st, (const int32_t *)w.loop.status,
                     d_info);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}
