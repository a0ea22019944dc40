// Sketch draw (Sec. 2.3) and the multi-column sketching routine RHSketch
// (Alg. 1) for gfx950.
//
// Randomness: Philox4x64-10 (Salmon et al., SC'11), key = (seed, stream),
// counter = (block, 0, 0, 0).  Stream 0: random signs (bit i%64 of word i/64);
// stream 1: one 64-bit key per coordinate, the l smallest (key, index) pairs
// give the sampled rows; stream 2: Box-Muller Gaussians for Omega.
#include "sketch_dev.h"

#include <algorithm>
#include <cmath>
#include <vector>

namespace {

constexpr uint64_t PM0 = 0xD2E7470EE14C6C93ull;
constexpr uint64_t PM1 = 0xCA5A826395121157ull;
constexpr uint64_t PW0 = 0x9E3779B97F4A7C15ull;
constexpr uint64_t PW1 = 0xBB67AE8584CAA73Bull;

__device__ __forceinline__ void philox(uint64_t x[4], uint64_t k0, uint64_t k1) {
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    if (r > 0) {
      k0 += PW0;
      k1 += PW1;
    }
    const uint64_t hi0 = __umul64hi(PM0, x[0]), lo0 = PM0 * x[0];
    const uint64_t hi1 = __umul64hi(PM1, x[2]), lo1 = PM1 * x[2];
    const uint64_t y0 = hi1 ^ x[1] ^ k0, y2 = hi0 ^ x[3] ^ k1;
    x[0] = y0;
    x[1] = lo1;
    x[2] = y2;
    x[3] = lo0;
  }
}

// signs: word w of stream 0 for w < nwords
__global__ void k_signs(uint64_t *out, int64_t nwords, uint64_t seed) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;  // philox block
  if (4 * b >= nwords) return;
  uint64_t x[4] = {(uint64_t)b, 0, 0, 0};
  philox(x, seed, 0);
  for (int w = 0; w < 4; ++w)
    if (4 * b + w < nwords) out[4 * b + w] = x[w];
}

// row keys: candidates with key <= thresh are appended (order irrelevant:
// the selection below sorts them).
__global__ void k_rowkeys(int64_t N, uint64_t seed, uint64_t thresh, int all,
                          unsigned long long *cnt, uint64_t *ckey, int32_t *cidx, int cap) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (4 * b >= N) return;
  uint64_t x[4] = {(uint64_t)b, 0, 0, 0};
  philox(x, seed, 1);
  for (int w = 0; w < 4; ++w) {
    const int64_t i = 4 * b + w;
    if (i < N && (all || x[w] <= thresh)) {
      const unsigned long long slot = atomicAdd(cnt, 1ull);
      if (slot < (unsigned long long)cap) {
        ckey[slot] = x[w];
        cidx[slot] = (int32_t)i;
      }
    }
  }
}

// One workgroup: bitonic sort of `cnt` (key, idx) pairs padded to P (power of
// two) by (key, idx); the first l indices are then sorted increasingly.
// LDS: key[P] (u64), idx[P] (i32), v[Pl] (i32).
__global__ void __launch_bounds__(1024) k_select_rows(const uint64_t *ckey, const int32_t *cidx,
                                                       int cnt, int P, int Pl, int l, int32_t *rows) {
  extern __shared__ unsigned char smem[];
  uint64_t *key = (uint64_t *)smem;
  int32_t *idx = (int32_t *)(key + P);
  int32_t *v = idx + P;
  for (int i = threadIdx.x; i < P; i += blockDim.x) {
    key[i] = i < cnt ? ckey[i] : ~0ull;
    idx[i] = i < cnt ? cidx[i] : 0x7fffffff;
  }
  __syncthreads();
  for (int k = 2; k <= P; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < P; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          const bool gt = key[i] > key[p] || (key[i] == key[p] && idx[i] > idx[p]);
          if (gt == up) {
            const uint64_t tk = key[i];
            key[i] = key[p];
            key[p] = tk;
            const int32_t ti = idx[i];
            idx[i] = idx[p];
            idx[p] = ti;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < Pl; i += blockDim.x) v[i] = i < l ? idx[i] : 0x7fffffff;
  __syncthreads();
  for (int k = 2; k <= Pl; k <<= 1) {
    for (int j = k >> 1; j > 0; j >>= 1) {
      for (int i = threadIdx.x; i < Pl; i += blockDim.x) {
        const int p = i ^ j;
        if (p > i) {
          const bool up = (i & k) == 0;
          if ((v[i] > v[p]) == up) {
            const int32_t t = v[i];
            v[i] = v[p];
            v[p] = t;
          }
        }
      }
      __syncthreads();
    }
  }
  for (int i = threadIdx.x; i < l; i += blockDim.x) rows[i] = v[i];
}

// Gaussian Omega: entry e = k + l*i (column-major, ld = l); one Philox block
// feeds entries 2b (words 0,1) and 2b+1 (words 2,3).
__global__ void k_gauss(double *om, int64_t count, uint64_t seed, double inv_sqrt_l_div) {
  const int64_t b = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (2 * b >= count) return;
  uint64_t x[4] = {(uint64_t)b, 0, 0, 0};
  philox(x, seed, 2);
  for (int h = 0; h < 2; ++h) {
    const int64_t e = 2 * b + h;
    if (e >= count) break;
    const double u1 = (double)((x[2 * h] >> 11) + 1ull) * 0x1.0p-53;
    const double u2 = (double)(x[2 * h + 1] >> 11) * 0x1.0p-53;
    const double g = sqrt(-2.0 * log(u1)) * cos(2.0 * M_PI * u2);
    om[e] = g / inv_sqrt_l_div;
  }
}

// ------------------------------------------------------------ RHSketch, SRHT
// Grid (gt, k): workgroup (g, c) transforms the row groups g, g+gt, ... of
// column c and accumulates its contribution to each of the l samples;
// part[c][g][q].
template <typename ST, typename AT, int QA>
__global__ void __launch_bounds__(SK_TPB) k_srht_cols(const ST *__restrict__ X, int64_t ldx, int64_t n,
                                                      int32_t m, int32_t l, int64_t ngroups, int gt,
                                                      const uint64_t *__restrict__ signs,
                                                      const int32_t *__restrict__ rows,
                                                      double *__restrict__ part, int aligned) {
  srht_cols_block<ST, AT, QA>(X, ldx, n, m, l, ngroups, gt, signs, rows, part, aligned, blockIdx.x,
                              blockIdx.y);
}

// Y[:, c] = [X_{1:m,c}; scale * sum_g part[c][g][:]]
template <typename ST>
__global__ void k_sketch_finish(const ST *__restrict__ X, int64_t ldx, int32_t m, int32_t l,
                                int gt, const double *__restrict__ part, double scale,
                                double *__restrict__ Y, int64_t ldy) {
  sketch_finish_one<ST>(X, ldx, m, l, gt, part, scale, Y, ldy,
                        blockIdx.x * blockDim.x + threadIdx.x, blockIdx.y);
}

// The same sum for few columns and many partial groups (gt > 64, e.g. the one
// column of an Arnoldi step): workgroup (b, c) sums rows q in [64 b, 64 b + 64)
// of column c, thread (qi, gs) the groups g = gs, gs + 16, ... (a 512-byte
// row of part per g), then the 16 slices in order; the last workgroups of
// each column copy the head rows.
constexpr int FW_Q = 64, FW_G = 16;
template <typename ST>
__global__ void __launch_bounds__(FW_Q * FW_G) k_sketch_finish_wide(
    const ST *__restrict__ X, int64_t ldx, int32_t m, int32_t l, int gt,
    const double *__restrict__ part, double scale, double *__restrict__ Y, int64_t ldy) {
  const int c = blockIdx.y;
  const int qb = (l + FW_Q - 1) / FW_Q;
  if ((int)blockIdx.x >= qb) {  // head rows
    for (int k = ((int)blockIdx.x - qb) * blockDim.x + threadIdx.x; k < m;
         k += (gridDim.x - qb) * blockDim.x)
      Y[(int64_t)c * ldy + k] = cvt_in<double>(X[(int64_t)c * ldx + k]);
    return;
  }
  __shared__ double red[FW_G][FW_Q];
  const int qi = threadIdx.x % FW_Q, gs = threadIdx.x / FW_Q;
  const int q = blockIdx.x * FW_Q + qi;
  const int qc = q < l ? q : l - 1;
  const double *p = part + (int64_t)c * gt * l + qc;
  double v = 0.0;
  int g = gs;
  for (; g + FW_G * 7 < gt; g += FW_G * 8) {
    double t[8];
#pragma unroll
    for (int b = 0; b < 8; ++b) t[b] = p[(int64_t)(g + FW_G * b) * l];
#pragma unroll
    for (int b = 0; b < 8; ++b) v += t[b];
  }
  for (; g < gt; g += FW_G) v += p[(int64_t)g * l];
  red[gs][qi] = v;
  __syncthreads();
  if (gs == 0 && q < l) {
    double sum = 0.0;
#pragma unroll
    for (int i = 0; i < FW_G; ++i) sum += red[i][qi];
    Y[(int64_t)c * ldy + m + q] = sum * scale;
  }
}

// ------------------------------------------------------------ RHSketch, Gaussian
// Split-K product  part[kc] = Omega[:, rows of chunk kc] X2[chunk, :]  on
// matrix cores (v_mfma_f64_16x16x4; float32 for low-precision storage, as the
// vector path computed in): 128 x 128 output tiles, so each chunk of Omega is
// read once per 128 columns of X2 and each chunk of X2 once per 128 rows of
// Omega; GMK-deep K steps staged in LDS, the next step's loads issued before
// this step's products.  Wave w owns tile rows 32 w .. 32 w + 31 (2 row
// blocks) and all 8 column blocks.
constexpr int GM = 128, GN = 128, GMK = 16;
template <typename CT> constexpr int gpad() {
  // row pitch of the LDS tiles: the 4 rows a product step reads (one per lane
  // group) fall on different halves of the banks
  return sizeof(CT) == 8 ? 16 : 32;
}
template <typename ST, typename CT>
__global__ void __launch_bounds__(256) k_gauss_mx(const double *__restrict__ om, int64_t ldo,
                                                  const ST *__restrict__ X, int64_t ldx, int32_t m,
                                                  int64_t ntail, int32_t l, int32_t k,
                                                  int64_t kchunk, double *__restrict__ part) {
  using Ops = PxOps<CT>;
  using acc_t = typename Ops::acc_t;
  constexpr int P = gpad<CT>();
  constexpr int NL = GMK * GM / 256;  // elements per thread and tile
  static_assert(GM == GN, "one staging pattern for both tiles");
  __shared__ CT As[GMK][GM + P];  // As[kk][q]   = Omega[q][chunk row kk]
  __shared__ CT Bs[GMK][GN + P];  // Bs[kk][col] = X2[chunk row kk][col]
  const int qt = blockIdx.x, ct = blockIdx.y, kc = blockIdx.z;
  const int tid = threadIdx.x, lane = tid & 63, w = tid >> 6;
  const int i16 = lane & 15, kq = lane >> 4;
  const int64_t k0 = (int64_t)kc * kchunk;
  const int64_t k1 = min(ntail, k0 + kchunk);
  acc_t acc[2][8];
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) acc[rb][cb][t] = (CT)0;
  // element e of a step: Omega row e % GM of chunk row e / GM (rows of Omega
  // contiguous), X2 chunk row e % GMK of column e / GMK (rows of X2 contiguous)
  CT ra[NL], rb_[NL];
  auto gload = [&](int64_t kk) {
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + 256 * i;
      const int64_t ki = kk + e / GM;
      const int q = qt * GM + e % GM;
      ra[i] = (ki < k1 && q < l) ? (CT)om[ki * ldo + q] : (CT)0;
      const int64_t ki2 = kk + e % GMK;
      const int col = ct * GN + e / GMK;
      rb_[i] = (ki2 < k1 && col < k) ? cvt_in<CT>(X[(int64_t)col * ldx + m + ki2]) : (CT)0;
    }
  };
  if (k0 < k1) gload(k0);
  for (int64_t kk = k0; kk < k1; kk += GMK) {
    __syncthreads();  // the previous step's tiles have been read
#pragma unroll
    for (int i = 0; i < NL; ++i) {
      const int e = tid + 256 * i;
      As[e / GM][e % GM] = ra[i];
      Bs[e % GMK][e / GMK] = rb_[i];
    }
    __syncthreads();
    if (kk + GMK < k1) gload(kk + GMK);
#pragma unroll
    for (int s4 = 0; s4 < GMK / 4; ++s4) {
      CT a[2];
#pragma unroll
      for (int rb = 0; rb < 2; ++rb) a[rb] = As[4 * s4 + kq][32 * w + 16 * rb + i16];
#pragma unroll
      for (int cb = 0; cb < 8; ++cb) {
        const CT bv = Bs[4 * s4 + kq][16 * cb + i16];
#pragma unroll
        for (int rb = 0; rb < 2; ++rb) acc[rb][cb] = Ops::mma(a[rb], bv, acc[rb][cb]);
      }
    }
  }
  // part layout: [col][kc][q]
  const int nkc = gridDim.z;
#pragma unroll
  for (int rb = 0; rb < 2; ++rb)
#pragma unroll
    for (int cb = 0; cb < 8; ++cb)
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int q = qt * GM + 32 * w + 16 * rb + Ops::di(kq, t);
        const int col = ct * GN + 16 * cb + i16;
        if (q < l && col < k) part[((int64_t)col * nkc + kc) * l + q] = (double)acc[rb][cb][t];
      }
}

// Y = [X head; scale * sum of the gt partial groups]: one thread per row,
// or, for more than 64 groups, the group sum spread over 16 threads per row
template <typename ST>
void launch_finish(const ST *X, int64_t ldx, int32_t m, int32_t l, int32_t k, int gt,
                   const double *part, double scale, double *Y, int64_t ldy, hipStream_t st) {
  if (gt > 64) {
    const int qb = (l + FW_Q - 1) / FW_Q, hb = (m + FW_Q * FW_G - 1) / (FW_Q * FW_G);
    hipLaunchKernelGGL((k_sketch_finish_wide<ST>), dim3(qb + hb, k), dim3(FW_Q * FW_G), 0, st, X,
                       ldx, m, l, gt, part, scale, Y, ldy);
  } else {
    hipLaunchKernelGGL((k_sketch_finish<ST>), dim3((m + l + 255) / 256, k), dim3(256), 0, st, X,
                       ldx, m, l, gt, part, scale, Y, ldy);
  }
}

template <typename ST>
int launch_typed(const rhqr_sketch_s *h, int64_t n, int32_t k, const ST *X, int64_t ldx,
                 double *Y, int64_t ldy, double *part, hipStream_t st) {
  const int32_t m = h->m, l = h->l;
  using CT = typename CompT<ST>::type;
  int gt = 1;
  size_t need = 0;
  sketch_tail_partials_size(h, k, &gt, &need);
  if (h->kind == RHQR_SKETCH_SRHT) {
    const int64_t ntiles = (n + TILE - 1) / TILE;
    const int aligned = ((uintptr_t)X % 16 == 0) && ((ldx * (int64_t)sizeof(ST)) % 16 == 0);
    const int64_t ngroups = (n + (int64_t)TILE * SK_TPW - 1) / ((int64_t)TILE * SK_TPW);
    // samples per thread: ceil(l / SK_TPB), rounded up to a power of two (l <= TILE)
    static_assert(8 * SK_TPB >= TILE, "at most 8 samples per thread");
    const int qa = l <= SK_TPB ? 1 : l <= 2 * SK_TPB ? 2 : l <= 4 * SK_TPB ? 4 : 8;
#define RHQR_SRHT_COLS(Q)                                                                    \
  RHQR_LAUNCH(RHQR_PROF_PRESKETCH, (k_srht_cols<ST, CT, Q>), dim3(gt, k), dim3(SK_TPB), 0, st, X, \
              ldx, n, m, l, ngroups, gt, h->d_signs, h->d_rows, part, aligned)
    switch (qa) {
      case 1: RHQR_SRHT_COLS(1); break;
      case 2: RHQR_SRHT_COLS(2); break;
      case 4: RHQR_SRHT_COLS(4); break;
      default: RHQR_SRHT_COLS(8); break;
    }
#undef RHQR_SRHT_COLS
    RHQR_HIP(hipGetLastError());
    launch_finish<ST>(X, ldx, m, l, k, gt, part, 1.0 / std::sqrt((double)l), Y, ldy, st);
  } else {
    const int64_t ntail = n - m;
    const int64_t kchunk = ((ntail + gt - 1) / gt + GMK - 1) / GMK * GMK;
    dim3 grid((l + GM - 1) / GM, (k + GN - 1) / GN, gt);
    RHQR_LAUNCH(RHQR_PROF_PRESKETCH, (k_gauss_mx<ST, CT>), grid, dim3(256), 0, st, h->d_omega,
                (int64_t)l, X, ldx, m, ntail, l, k, kchunk, part);
    launch_finish<ST>(X, ldx, m, l, k, gt, part, 1.0, Y, ldy, st);
  }
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

}  // namespace

// Number of partial-sum groups per column and the partial buffer size.
int sketch_tail_partials_size(const rhqr_sketch_s *h, int32_t k, int *gt_out, size_t *bytes_out) {
  int gt;
  if (h->kind == RHQR_SKETCH_SRHT) {
    const int64_t ngroups = (h->n + (int64_t)TILE * SK_TPW - 1) / ((int64_t)TILE * SK_TPW);
    const int64_t target = std::max<int64_t>(1, 2048 / std::max<int32_t>(k, 1));
    gt = (int)std::min<int64_t>(ngroups, target);
  } else {
    const int64_t ntail = h->n - h->m;
    const int64_t tiles = (int64_t)((h->l + GM - 1) / GM) * ((k + GN - 1) / GN);
    const int64_t target = std::max<int64_t>(1, 512 / tiles);  // about 2 workgroups per unit
    gt = (int)std::max<int64_t>(1, std::min<int64_t>(target, (ntail + 4095) / 4096));
  }
  *gt_out = gt;
  *bytes_out = align_up((size_t)k * gt * h->l * sizeof(double));
  return 0;
}

size_t sketch_ws_bytes(const rhqr_sketch_s *h, int32_t k) {
  int gt;
  size_t b;
  sketch_tail_partials_size(h, k, &gt, &b);
  return b;
}

int launch_sketch(const rhqr_sketch_s *h, int dtype, int64_t n, int32_t k, const void *X,
                  int64_t ldx, double *Y, int64_t ldy, void *ws, size_t ws_bytes, hipStream_t st) {
  if (ws_bytes < sketch_ws_bytes(h, k)) return RHQR_ERR_WORKSPACE;
  double *part = (double *)ws;
  switch (dtype) {
    case RHQR_F64: return launch_typed<double>(h, n, k, (const double *)X, ldx, Y, ldy, part, st);
    case RHQR_F32: return launch_typed<float>(h, n, k, (const float *)X, ldx, Y, ldy, part, st);
    case RHQR_F16: return launch_typed<__half>(h, n, k, (const __half *)X, ldx, Y, ldy, part, st);
    case RHQR_BF16:
      return launch_typed<__hip_bfloat16>(h, n, k, (const __hip_bfloat16 *)X, ldx, Y, ldy, part, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

// ================================================================ C ABI
extern "C" int rhqr_sketch_create(int kind, int64_t n, int32_t m, int32_t l, uint64_t seed,
                                  const double *d_omega, int64_t ld_omega, void *stream,
                                  rhqr_sketch_t *out) {
  if (kind != RHQR_SKETCH_SRHT && kind != RHQR_SKETCH_GAUSS) return -1;
  if (n < 2) return -2;
  if (m < 0 || m >= n) return -3;  // m = 0: Omega on every row (trimRHQR)
  int64_t N = 1;
  while (N < n) N <<= 1;
  if (l < 1 || (kind == RHQR_SKETCH_SRHT && (l > N || l > TILE))) return -4;
  if (kind == RHQR_SKETCH_GAUSS && d_omega && ld_omega < l) return -7;
  if (!out) return -9;
  if (N > ((int64_t)1 << 31)) return -2;
  hipStream_t st = (hipStream_t)stream;
  rhqr_sketch_s *h = new rhqr_sketch_s();
  h->kind = kind;
  h->n = n;
  h->m = m;
  h->l = l;
  h->seed = seed;
  h->N = N;
  h->d_signs = nullptr;
  h->d_rows = nullptr;
  h->d_omega = nullptr;
  if (hipGetDevice(&h->device) != hipSuccess) {
    delete h;
    return RHQR_ERR_HIP;
  }
  auto fail = [&](int code) {
    rhqr_sketch_destroy(h);
    return code;
  };
  if (kind == RHQR_SKETCH_SRHT) {
    const int64_t nw = (N + 63) / 64;
    if (hipMalloc(&h->d_signs, nw * sizeof(uint64_t)) != hipSuccess) return fail(RHQR_ERR_HIP);
    if (hipMalloc(&h->d_rows, (size_t)l * sizeof(int32_t)) != hipSuccess) return fail(RHQR_ERR_HIP);
    const int64_t nb = (nw + 3) / 4;
    hipLaunchKernelGGL(k_signs, dim3((nb + 255) / 256), dim3(256), 0, st, h->d_signs, nw, seed);
    if (hipGetLastError() != hipSuccess) return fail(RHQR_ERR_HIP);
    // selection of the l smallest keys: threshold draw, then a sort
    const int cap = 8192;
    uint64_t *ckey = nullptr;
    int32_t *cidx = nullptr;
    unsigned long long *cnt = nullptr;
    if (hipMalloc(&ckey, cap * sizeof(uint64_t)) != hipSuccess) return fail(RHQR_ERR_HIP);
    if (hipMalloc(&cidx, cap * sizeof(int32_t)) != hipSuccess) {
      (void)hipFree(ckey);
      return fail(RHQR_ERR_HIP);
    }
    if (hipMalloc(&cnt, sizeof(unsigned long long)) != hipSuccess) {
      (void)hipFree(ckey);
      (void)hipFree(cidx);
      return fail(RHQR_ERR_HIP);
    }
    double expect = l + 10.0 * std::sqrt((double)l) + 64.0;
    int rc = RHQR_OK;
    unsigned long long hc = 0;
    for (int attempt = 0; attempt < 8; ++attempt) {
      const int all = expect >= (double)N ? 1 : 0;
      if (all && N > cap) {
        rc = RHQR_ERR_UNSUPPORTED;
        break;
      }
      const long double frac = all ? 1.0L : (long double)expect / (long double)N;
      const uint64_t thresh = all ? ~0ull : (uint64_t)(frac * 18446744073709551616.0L);
      if (hipMemsetAsync(cnt, 0, sizeof(unsigned long long), st) != hipSuccess) { rc = RHQR_ERR_HIP; break; }
      const int64_t nb4 = (N + 3) / 4;
      hipLaunchKernelGGL(k_rowkeys, dim3((nb4 + 255) / 256), dim3(256), 0, st, N, seed, thresh,
                         all, cnt, ckey, cidx, cap);
      if (hipGetLastError() != hipSuccess) { rc = RHQR_ERR_HIP; break; }
      if (hipMemcpyAsync(&hc, cnt, sizeof(hc), hipMemcpyDeviceToHost, st) != hipSuccess ||
          hipStreamSynchronize(st) != hipSuccess) { rc = RHQR_ERR_HIP; break; }
      if (hc >= (unsigned long long)l && hc <= (unsigned long long)cap) break;
      if (hc > (unsigned long long)cap) expect *= 0.5; else expect *= 2.0;
      if (attempt == 7) rc = RHQR_ERR_UNSUPPORTED;
    }
    if (rc == RHQR_OK) {
      int P = 1;
      while (P < (int)hc) P <<= 1;
      int Pl = 1;
      while (Pl < l) Pl <<= 1;
      const size_t shm = (size_t)P * 8 + (size_t)P * 4 + (size_t)Pl * 4;
      hipLaunchKernelGGL(k_select_rows, dim3(1), dim3(1024), shm, st, ckey, cidx, (int)hc, P, Pl,
                         l, h->d_rows);
      if (hipGetLastError() != hipSuccess || hipStreamSynchronize(st) != hipSuccess) rc = RHQR_ERR_HIP;
    }
    (void)hipFree(ckey);
    (void)hipFree(cidx);
    (void)hipFree(cnt);
    if (rc != RHQR_OK) return fail(rc);
  } else {
    const int64_t ntail = n - m;
    const int64_t count = (int64_t)l * ntail;
    if (hipMalloc(&h->d_omega, (size_t)count * sizeof(double)) != hipSuccess) return fail(RHQR_ERR_HIP);
    if (d_omega) {
      if (hipMemcpy2DAsync(h->d_omega, (size_t)l * sizeof(double), d_omega,
                           (size_t)ld_omega * sizeof(double), (size_t)l * sizeof(double),
                           (size_t)ntail, hipMemcpyDeviceToDevice, st) != hipSuccess)
        return fail(RHQR_ERR_HIP);
    } else {
      const int64_t nb = (count + 1) / 2;
      hipLaunchKernelGGL(k_gauss, dim3((nb + 255) / 256), dim3(256), 0, st, h->d_omega, count,
                         seed, std::sqrt((double)l));
      if (hipGetLastError() != hipSuccess) return fail(RHQR_ERR_HIP);
    }
    if (hipStreamSynchronize(st) != hipSuccess) return fail(RHQR_ERR_HIP);
  }
  *out = h;
  return RHQR_OK;
}

extern "C" int rhqr_sketch_destroy(rhqr_sketch_t h) {
  if (!h) return -1;
  if (h->d_signs) (void)hipFree(h->d_signs);
  if (h->d_rows) (void)hipFree(h->d_rows);
  if (h->d_omega) (void)hipFree(h->d_omega);
  delete h;
  return RHQR_OK;
}

extern "C" int rhqr_sketch_get(rhqr_sketch_t h, uint64_t *h_signs, int32_t *h_rows, double *h_omega) {
  if (!h) return -1;
  if (h_signs && h->d_signs)
    RHQR_HIP(hipMemcpy(h_signs, h->d_signs, ((h->N + 63) / 64) * sizeof(uint64_t), hipMemcpyDeviceToHost));
  if (h_rows && h->d_rows)
    RHQR_HIP(hipMemcpy(h_rows, h->d_rows, (size_t)h->l * sizeof(int32_t), hipMemcpyDeviceToHost));
  if (h_omega && h->d_omega)
    RHQR_HIP(hipMemcpy(h_omega, h->d_omega, (size_t)h->l * (h->n - h->m) * sizeof(double),
                       hipMemcpyDeviceToHost));
  return RHQR_OK;
}

extern "C" int rhqr_sketch_info(rhqr_sketch_t h, int64_t *n, int32_t *m, int32_t *l, int64_t *N,
                                int32_t *kind) {
  if (!h) return -1;
  if (n) *n = h->n;
  if (m) *m = h->m;
  if (l) *l = h->l;
  if (N) *N = h->N;
  if (kind) *kind = h->kind;
  return RHQR_OK;
}

extern "C" size_t rhqr_sketch_workspace_size(rhqr_sketch_t h, int32_t k) {
  if (!h || k < 1) return 0;
  return sketch_ws_bytes(h, k);
}

extern "C" int rhqr_sketch(rhqr_sketch_t h, int dtype, int64_t n, int32_t k, const void *d_X,
                           int64_t ldx, double *d_Y, int64_t ldy, void *d_ws, size_t ws_bytes,
                           void *stream) {
  if (!h) return -1;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -2;
  if (n != h->n) return -3;
  if (k < 1) return -4;
  if (!d_X) return -5;
  if (ldx < n) return -6;
  if (!d_Y) return -7;
  if (ldy < h->l + h->m) return -8;
  if (!d_ws) return -9;
  return launch_sketch(h, dtype, n, k, d_X, ldx, d_Y, ldy, d_ws, ws_bytes, (hipStream_t)stream);
}
