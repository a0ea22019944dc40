// Batched left-looking RHQR (Alg. 4 with RHVector, Alg. 2): many independent
// problems, each with its own W (n_p x m_p), sketch (SRHT or Gaussian, one
// kind per batch) and outputs, factored
// by one fixed sequence of launches that allocates nothing, synchronises with
// nothing on the host and can be captured once in a hipGraph and replayed.
//
// Problems are ordered by decreasing m, so the problems still active at column
// j (m_p > j) are a prefix of that order.  Per column j the sequence is one
// tall launch, one reduction launch and one step launch over all active
// problems; every workgroup finds its (problem, local block) in a block map
// built at creation, then runs exactly the single-problem device code
// (colstep.h, sketch_dev.h) on that problem's descriptor.  A problem's result
// is therefore bitwise the one rhqr_factor (column schedule) gives it.
#include "colstep.h"
#include "sketch_dev.h"

#include <algorithm>
#include <cmath>
#include <numeric>
#include <vector>

namespace {

struct BlockMap {
  int32_t p, local;
};

// pre-sketch of one problem's m columns
struct SketchJob {
  const void *X;
  int64_t ldx, n;
  int32_t m, l;
  int64_t ngroups;
  int32_t gt, aligned;
  const uint64_t *signs;
  const int32_t *rows;
  double *part;
  double *Z;
  int64_t ldz;
  double scale;
};

__global__ void kb_init(const ColProblem *__restrict__ P) {
  const ColProblem &Q = P[blockIdx.x];
  const int32_t m = Q.m;
  for (int e = threadIdx.x; e < m * m; e += blockDim.x)
    Q.T[(e % m) + (int64_t)(e / m) * Q.ldt] = 0.0;
  if (threadIdx.x < 4) Q.status[threadIdx.x] = 0;
}

template <typename ST, typename AT, int QA>
__global__ void __launch_bounds__(SK_TPB) kb_srht_cols(const SketchJob *__restrict__ J,
                                                       const BlockMap *__restrict__ map) {
  const BlockMap b = map[blockIdx.x];
  const SketchJob &s = J[b.p];
  srht_cols_block<ST, AT, QA>((const ST *)s.X, s.ldx, s.n, s.m, s.l, s.ngroups, s.gt, s.signs,
                              s.rows, s.part, s.aligned, b.local % s.gt, b.local / s.gt);
}

template <typename ST>
__global__ void kb_sketch_finish(const SketchJob *__restrict__ J, const BlockMap *__restrict__ cmap) {
  const BlockMap b = cmap[blockIdx.x];
  const SketchJob &s = J[b.p];
  sketch_finish_one<ST>((const ST *)s.X, s.ldx, s.m, s.l, s.gt, s.part, s.scale, s.Z, s.ldz,
                        blockIdx.y * blockDim.x + threadIdx.x, b.local);
}

// 256-thread tall workgroups: several per compute unit, so one workgroup's
// transform overlaps the others' streaming (the problems are small); at least
// three per compute unit (the 2-byte types' 16 values per thread sit at the
// register budget of three)
constexpr int BATCH_TPB = 256;

template <typename ST, int TPW>
__global__ void __launch_bounds__(BATCH_TPB, 3) kb_tall(const ColProblem *__restrict__ P,
                                                     const BlockMap *__restrict__ map, int32_t j,
                                                     int32_t p0) {
  const BlockMap b = map[blockIdx.x];
  tall_block<ST, RHQR_SKETCH_SRHT, TPW, BATCH_TPB>(P[b.p], j, p0, b.local);
}

// Gaussian sketches: the tall workgroups of the single-problem path (1024
// threads; the Gaussian partial products assume them)
template <typename ST, int TPW>
__global__ void __launch_bounds__(1024) kb_tall_gauss(const ColProblem *__restrict__ P,
                                                      const BlockMap *__restrict__ map, int32_t j,
                                                      int32_t p0) {
  const BlockMap b = map[blockIdx.x];
  tall_block<ST, RHQR_SKETCH_GAUSS, TPW, 1024>(P[b.p], j, p0, b.local);
}

template <typename ST>
__global__ void __launch_bounds__(256) kb_red(const ColProblem *__restrict__ P,
                                              const BlockMap *__restrict__ map, int32_t j) {
  const BlockMap b = map[blockIdx.x];
  const ColProblem &Q = P[b.p];
  red_block<ST, RHQR_SKETCH_SRHT, 4>(Q, j, j + 1 < Q.m, b.local);
}

__global__ void __launch_bounds__(1024) kb_fin(const ColProblem *__restrict__ P, int32_t j, int fg) {
  const int p = blockIdx.x / fg, local = blockIdx.x % fg;
  const ColProblem &Q = P[p];
  fin_block(Q, j, j + 1 < Q.m, local, fg);
}

// ---- blocked schedule, per problem as in the single-problem path
// (run_blocked_typed): panels of `panel` columns, optionally grouped in outer
// panels of `outer`; before a panel at J, with the reflectors K0..J-1: store
// u_{J-1}, G = S_{<J}^t Z_panel, C = rows K0..J-1 of T^t G, then
// W_panel -= U_{K0:J} C.  A problem's panel has nb = min(width, m - J)
// columns; C has row pitch panel_width(nb) (8, 16 or 32), as in the single
// path, and is m x 32 per problem.
constexpr int BATCH_MAXPB = 32;
constexpr int SCALE_CH = 64;  // workgroups per problem in kb_scale_col

template <typename ST>
__global__ void kb_scale_col(const ColProblem *__restrict__ P, int32_t cidx) {
  const ColProblem &Q = P[blockIdx.x];
  ST *col = (ST *)Q.W + (int64_t)cidx * Q.ldw;
  const double a = Q.ia[cidx];
  const int64_t stride = (int64_t)gridDim.y * blockDim.x;
  for (int64_t i = Q.m + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < Q.n; i += stride) {
    col[i] = cvt_out<ST>(cvt_in<double>(col[i]) * a);  // raw values in place
  }
}

__global__ void __launch_bounds__(1024) kb_pgram(const ColProblem *__restrict__ P, int32_t J,
                                                 int32_t width, int per) {
  const int p = blockIdx.x / per, local = blockIdx.x % per;
  const ColProblem &Q = P[p];
  const int32_t nb = Q.m - J < width ? Q.m - J : width;
  pgram_block(Q.l + Q.m, J, nb, Q.S, Q.lds, Q.Z, Q.ldz, Q.G, local);
}

__global__ void __launch_bounds__(PTRI_WAVES * 64) kb_ptri(const ColProblem *__restrict__ P,
                                                          int32_t K0, int32_t J, int32_t width,
                                                          int per) {
  const int p = blockIdx.x / per, local = blockIdx.x % per;
  const ColProblem &Q = P[p];
  const int32_t nb = Q.m - J < width ? Q.m - J : width;
  ptri_wave(K0, J, nb, panel_width(nb), Q.T, Q.ldt, Q.G, Q.C,
            local * PTRI_WAVES + (threadIdx.x >> 6), blockIdx.y);
}

// workgroups per compute unit kb_panel is built for: those of the matrix-core
// update, except for 2-byte storage, whose vector-unit update of wide panels
// would spill at that register budget
template <typename ST> constexpr int kb_panel_min_wg() { return sizeof(ST) == 2 ? 1 : px_min_wg<ST>(); }

template <typename ST>
__global__ void __launch_bounds__(PANEL_TPB, kb_panel_min_wg<ST>()) kb_panel(const ColProblem *__restrict__ P,
                                                      const BlockMap *__restrict__ map, int32_t K0,
                                                      int32_t J, int32_t width) {
  const BlockMap b = map[blockIdx.x];
  const ColProblem &Q = P[b.p];
  const int32_t nb = Q.m - J < width ? Q.m - J : width;
  if (nb <= 0) return;  // the problem ended before this panel (whole workgroup)
  // the same choice of units and arithmetic as the single-problem update
  static_assert(PANEL_TPB == PX_WAVES * 64, "one panel workgroup layout for both units");
  ST *W = (ST *)Q.W;
  const int pw = panel_width(nb);
  if (Q.aligned && nb > PX_MIN_NB && nb <= 16) {
    panel_mx_block<ST, 16>(W, Q.ldw, W + (int64_t)J * Q.ldw, Q.ldw, false, Q.n, Q.m, K0, J, nb, pw,
                           Q.C, b.local);
  } else if (Q.aligned && nb > PX_MIN_NB) {
    panel_mx_block<ST, 32>(W, Q.ldw, W + (int64_t)J * Q.ldw, Q.ldw, false, Q.n, Q.m, K0, J, nb, pw,
                           Q.C, b.local);
  } else if (pw == 8) {
    panel_block<ST, 8>(W, Q.ldw, Q.n, Q.m, K0, J, nb, Q.C, Q.aligned, b.local, J);
  } else if (pw == 16) {
    panel_block<ST, 16>(W, Q.ldw, Q.n, Q.m, K0, J, nb, Q.C, Q.aligned, b.local, J);
  } else {
    panel_block<ST, 32>(W, Q.ldw, Q.n, Q.m, K0, J, nb, Q.C, Q.aligned, b.local, J);
  }
}

// last column stored as u = raw / alpha, head block of U written from S
template <typename ST>
__global__ void kb_finish(const ColProblem *__restrict__ P) {
  const ColProblem &Q = P[blockIdx.x];
  ST *W = (ST *)Q.W;
  const int32_t m = Q.m, cidx = m - 1;
  const double a = Q.ia[cidx];
  ST *col = W + (int64_t)cidx * Q.ldw;
  const int64_t stride = (int64_t)gridDim.y * blockDim.x;
  for (int64_t i = m + (int64_t)blockIdx.y * blockDim.x + threadIdx.x; i < Q.n; i += stride) {
    col[i] = cvt_out<ST>(cvt_in<double>(col[i]) * a);  // raw values in place
  }
  for (int64_t e = (int64_t)blockIdx.y * blockDim.x + threadIdx.x; e < (int64_t)m * m; e += stride) {
    const int k = (int)(e % m), c = (int)(e / m);
    W[k + (int64_t)c * Q.ldw] = cvt_out<ST>(Q.S[k + (int64_t)c * Q.lds]);
  }
}

constexpr int FINISH_CH = 64;  // workgroups per problem in kb_finish

// tall workgroups cover TPW transform tiles: two for 2-byte types (16-byte
// loads need eight rows per thread), one otherwise
inline int batch_tpw(int dtype) { return dtype_size(dtype) == 2 ? 2 : 1; }

struct Layout {
  // sorted order and per-problem geometry
  std::vector<int32_t> order;
  std::vector<int64_t> nparts, gred, gt, ngroups, npanel, qblocks, qgroups;
  std::vector<int32_t> qtiles, qkp;
  int64_t qblocks_total = 0;
  int32_t qtiles_max = 0;
  // prefix sums over the sorted problems
  std::vector<int64_t> tall_start, red_start, sk_start, col_start, pan_start;
  size_t head_bytes = 0, total = 0;
  std::vector<size_t> off;  // per sorted problem: start of its region
  size_t off_probs = 0, off_jobs = 0, off_tall = 0, off_red = 0, off_sk = 0, off_col = 0,
         off_pan = 0, off_qjobs = 0, off_qmap = 0;
};

size_t problem_bytes(const rhqr_sketch_s *h, int dtype) {
  const int32_t m = h->m, L = h->l + h->m;
  int gt;
  size_t skb;
  sketch_tail_partials_size(h, m, &gt, &skb);
  return align_up(loop_ws_bytes(h->kind, dtype, h->n, m, h->l)) +
         align_up(sizeof(double) * (size_t)L * m) + align_up(skb) +
         2 * align_up(sizeof(double) * (size_t)m * BATCH_MAXPB) +
         align_up(sizeof(double) * (size_t)m * m) + thin_q_bytes(m);  // thin Q: Mq, split coefficients
}

// panel-update workgroups of one problem (rows from m rounded down to the
// vector width): enough for every layout kb_panel may take (matrix cores,
// vector units with 8-, 16- or 32-column panels; each workgroup returns
// beyond its own last row)
template <typename ST> int64_t panel_groups_typed(int64_t n, int32_t m) {
  auto g = [&](int vec) {
    const int64_t mb0 = m - (m % vec);
    return (n - mb0 + (int64_t)PANEL_TPB * vec - 1) / ((int64_t)PANEL_TPB * vec);
  };
  int64_t r = panel_mx_groups(n, m, (int)sizeof(ST));
  r = std::max(r, g(panel_vec<ST, 8>()));
  r = std::max(r, g(panel_vec<ST, 16>()));
  return std::max(r, g(panel_vec<ST, 32>()));
}

int64_t panel_groups(int64_t n, int32_t m, int dtype) {
  switch (dtype) {
    case RHQR_F64: return panel_groups_typed<double>(n, m);
    case RHQR_F32: return panel_groups_typed<float>(n, m);
    case RHQR_F16: return panel_groups_typed<__half>(n, m);
    default: return panel_groups_typed<__hip_bfloat16>(n, m);
  }
}

int plan(const rhqr_problem *probs, int32_t count, int dtype, Layout *o) {
  const int tpw = batch_tpw(dtype);
  o->order.resize(count);
  std::iota(o->order.begin(), o->order.end(), 0);
  std::stable_sort(o->order.begin(), o->order.end(), [&](int a, int b) {
    return probs[a].sketch->m > probs[b].sketch->m;
  });
  o->nparts.resize(count);
  o->gred.resize(count);
  o->gt.resize(count);
  o->ngroups.resize(count);
  o->npanel.resize(count);
  o->qblocks.resize(count);
  o->qgroups.resize(count);
  o->qtiles.resize(count);
  o->qkp.resize(count);
  o->pan_start.assign(count + 1, 0);
  o->tall_start.assign(count + 1, 0);
  o->red_start.assign(count + 1, 0);
  o->sk_start.assign(count + 1, 0);
  o->col_start.assign(count + 1, 0);
  for (int s = 0; s < count; ++s) {
    const rhqr_sketch_s *h = probs[o->order[s]].sketch;
    int gt;
    size_t skb;
    sketch_tail_partials_size(h, h->m, &gt, &skb);
    o->nparts[s] = (h->n + (int64_t)TILE * tpw - 1) / ((int64_t)TILE * tpw);
    o->gred[s] = (h->m + RED_CHUNK - 1) / RED_CHUNK + (h->l + RED_CHUNK - 1) / RED_CHUNK;
    o->gt[s] = gt;
    o->ngroups[s] = (h->n + (int64_t)TILE * SK_TPW - 1) / ((int64_t)TILE * SK_TPW);
    o->tall_start[s + 1] = o->tall_start[s] + o->nparts[s];
    o->red_start[s + 1] = o->red_start[s] + o->gred[s];
    // the SRHT pre-sketch runs as blocks of one launch; a Gaussian batch
    // pre-sketches problem by problem (the split-K product of rhqr_sketch)
    o->sk_start[s + 1] = o->sk_start[s] + (h->kind == RHQR_SKETCH_SRHT ? (int64_t)h->m * gt : 0);
    o->col_start[s + 1] = o->col_start[s] + h->m;
    o->npanel[s] = panel_groups(h->n, h->m, dtype);
    o->qblocks[s] = thin_q_tail_blocks(dtype, h->n, h->m, &o->qtiles[s], &o->qgroups[s], &o->qkp[s]);
    o->qblocks_total += o->qblocks[s];
    o->qtiles_max = std::max(o->qtiles_max, o->qtiles[s]);
    o->pan_start[s + 1] = o->pan_start[s] + o->npanel[s];
  }
  if (o->tall_start[count] > INT32_MAX || o->sk_start[count] > INT32_MAX ||
      o->pan_start[count] > INT32_MAX || o->qblocks_total > INT32_MAX)
    return RHQR_ERR_UNSUPPORTED;
  size_t b = 0;
  auto take = [&](size_t bytes) {
    const size_t r = b;
    b += align_up(bytes);
    return r;
  };
  o->off_probs = take(sizeof(ColProblem) * count);
  o->off_jobs = take(sizeof(SketchJob) * count);
  o->off_tall = take(sizeof(BlockMap) * o->tall_start[count]);
  o->off_red = take(sizeof(BlockMap) * o->red_start[count]);
  o->off_sk = take(sizeof(BlockMap) * o->sk_start[count]);
  o->off_col = take(sizeof(BlockMap) * o->col_start[count]);
  o->off_pan = take(sizeof(BlockMap) * o->pan_start[count]);
  o->off_qjobs = take(sizeof(ThinQJob) * count);
  o->off_qmap = take(sizeof(ThinQBlock) * o->qblocks_total);
  o->head_bytes = b;
  o->off.resize(count);
  for (int s = 0; s < count; ++s) o->off[s] = take(problem_bytes(probs[o->order[s]].sketch, dtype));
  o->total = b;
  return RHQR_OK;
}

int check_problems(const rhqr_problem *probs, int32_t count, int dtype) {
  if (!probs) return -1;
  if (count < 1) return -2;
  if (dtype < RHQR_F64 || dtype > RHQR_BF16) return -3;
  for (int32_t i = 0; i < count; ++i) {
    const rhqr_problem &q = probs[i];
    const rhqr_sketch_s *h = q.sketch;
    if (!h || (h->kind != RHQR_SKETCH_SRHT && h->kind != RHQR_SKETCH_GAUSS)) return -1;
    if (h->kind != probs[0].sketch->kind) return -1;  // one sketch kind per batch
    if (h->m < 1 || h->m > MAXM || h->l > 4096) return -1;
    if (!q.d_W || q.ldw < h->n) return -1;
    if (!q.d_S || q.lds < h->l + h->m) return -1;
    if (!q.d_T || q.ldt < h->m) return -1;
    if (!q.d_R || q.ldr < h->m) return -1;
  }
  return RHQR_OK;
}

}  // namespace

struct rhqr_batch_s {
  int dtype = 0, count = 0, maxm = 0, tpw = 1, qa = 1, maxL = 0;
  int kind = RHQR_SKETCH_SRHT;     // every problem's sketch kind
  std::vector<const rhqr_sketch_s *> hs;  // per problem (sorted): its sketch handle,
  std::vector<double *> skpart, zs;       //   pre-sketch partials and Z (Gaussian batches)
  std::vector<size_t> skbytes;
  int panel = 0;                  // 0: column schedule; 2 .. 32: blocked
  int outer = 0;                  // 0: one level; else outer panels (a multiple of panel)
  std::vector<int32_t> order;     // sorted position -> caller index
  std::vector<int32_t> ms;        // m of each sorted problem (decreasing)
  std::vector<int64_t> tall_start, red_start, pan_start;
  int64_t sk_blocks = 0, cols = 0;
  std::vector<ColProblem> hp;     // host copy of the descriptors (sorted)
  std::vector<double *> mq;       // per problem (sorted): thin-Q scratch (m x m float64)
  std::vector<void *> qmf;        //   and the split coefficients of the 2-byte thin Q
  // batched thin Q: the per-problem jobs without their Q (filled per call in
  // a pinned staging table, uploaded to d_qjobs), the tail-workgroup map
  std::vector<ThinQJob> qjob;
  ThinQJob *h_qjobs = nullptr, *d_qjobs = nullptr;
  ThinQBlock *d_qmap = nullptr;
  int64_t qblocks = 0;
  int32_t qtiles_max = 0;
  hipEvent_t qev = nullptr;  // the last upload of the staging table
  bool qev_pending = false;
  ColProblem *d_probs = nullptr;
  SketchJob *d_jobs = nullptr;
  BlockMap *d_tall = nullptr, *d_red = nullptr, *d_sk = nullptr, *d_col = nullptr,
           *d_pan = nullptr;
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

namespace {

// active problems at column j: m_p > j (a prefix of the sorted order)
int active(const rhqr_batch_s *b, int32_t j) {
  return (int)(std::partition_point(b->ms.begin(), b->ms.end(), [j](int32_t m) { return m > j; }) -
               b->ms.begin());
}

template <typename ST>
int enqueue_typed(rhqr_batch_s *b, hipStream_t st) {
  using AT = typename CompT<ST>::type;
  hipLaunchKernelGGL(kb_init, dim3(b->count), dim3(256), 0, st, b->d_probs);
  RHQR_HIP(hipGetLastError());
  const bool gauss = b->kind == RHQR_SKETCH_GAUSS;
  if (gauss) {
    // Z = Psi W per problem: the single-problem pre-sketch (split-K product
    // on matrix cores and its finish), so Z equals rhqr_factor's bitwise
    for (int s = 0; s < b->count; ++s) {
      const ColProblem &P = b->hp[s];
      const int rc = launch_sketch(b->hs[s], b->dtype, P.n, P.m, P.W, P.ldw, b->zs[s],
                                   P.ldz, b->skpart[s], b->skbytes[s], st);
      if (rc) return rc;
    }
  } else {
  switch (b->qa) {
    case 1:
      hipLaunchKernelGGL((kb_srht_cols<ST, AT, 1>), dim3(b->sk_blocks), dim3(SK_TPB), 0, st, b->d_jobs, b->d_sk);
      break;
    case 2:
      hipLaunchKernelGGL((kb_srht_cols<ST, AT, 2>), dim3(b->sk_blocks), dim3(SK_TPB), 0, st, b->d_jobs, b->d_sk);
      break;
    case 4:
      hipLaunchKernelGGL((kb_srht_cols<ST, AT, 4>), dim3(b->sk_blocks), dim3(SK_TPB), 0, st, b->d_jobs, b->d_sk);
      break;
    default:
      hipLaunchKernelGGL((kb_srht_cols<ST, AT, 8>), dim3(b->sk_blocks), dim3(SK_TPB), 0, st, b->d_jobs, b->d_sk);
  }
  RHQR_HIP(hipGetLastError());
  hipLaunchKernelGGL((kb_sketch_finish<ST>), dim3(b->cols, (b->maxL + 255) / 256), dim3(256), 0, st,
                     b->d_jobs, b->d_col);
  RHQR_HIP(hipGetLastError());
  }
  // W_{:, J:J+width} -= U_{:, K0:J} C for every problem still active at J
  auto apply = [&](int32_t K0, int32_t J, int32_t width) -> int {
    const int a = active(b, J);
    hipLaunchKernelGGL((kb_scale_col<ST>), dim3(a, SCALE_CH), dim3(256), 0, st, b->d_probs, J - 1);
    RHQR_HIP(hipGetLastError());
    const int pg = (J * width + 15) / 16;
    hipLaunchKernelGGL(kb_pgram, dim3(a * pg), dim3(1024), 0, st, b->d_probs, J, width, pg);
    RHQR_HIP(hipGetLastError());
    const int pt = (J + PTRI_WAVES - 1) / PTRI_WAVES;
    hipLaunchKernelGGL(kb_ptri, dim3(a * pt, panel_width(width)), dim3(PTRI_WAVES * 64), 0, st,
                       b->d_probs, K0, J, width, pt);
    RHQR_HIP(hipGetLastError());
    hipLaunchKernelGGL((kb_panel<ST>), dim3(b->pan_start[a]), dim3(PANEL_TPB), 0, st, b->d_probs,
                       b->d_pan, K0, J, width);
    RHQR_HIP(hipGetLastError());
    return RHQR_OK;
  };
  // the loop of run_blocked_typed over the largest m (column schedule: one panel)
  const int pb = b->panel >= 2 ? b->panel : b->maxm;
  const int ob = b->outer > pb ? b->outer : pb;
  for (int32_t J0 = 0; J0 < b->maxm; J0 += ob) {
    if (J0 > 0) {
      const int rc = apply(0, J0, ob);
      if (rc) return rc;
    }
    for (int32_t J = J0; J < J0 + ob && J < b->maxm; J += pb) {
      if (J > J0) {
        const int rc = apply(J0, J, pb);
        if (rc) return rc;
      }
      const int32_t jend = std::min(std::min(J + pb, J0 + ob), b->maxm);
      for (int32_t j = J; j < jend; ++j) {
        const int a = active(b, j);
        if (j >= 1) {
          constexpr int TPW = sizeof(ST) == 2 ? 2 : 1;  // = batch_tpw(dtype)
          if (gauss)
            hipLaunchKernelGGL((kb_tall_gauss<ST, TPW>), dim3(b->tall_start[a]), dim3(1024), 0, st,
                               b->d_probs, b->d_tall, j, J);
          else
            hipLaunchKernelGGL((kb_tall<ST, TPW>), dim3(b->tall_start[a]), dim3(BATCH_TPB), 0, st,
                               b->d_probs, b->d_tall, j, J);
          RHQR_HIP(hipGetLastError());
        }
        hipLaunchKernelGGL((kb_red<ST>), dim3(b->red_start[a]), dim3(256), 0, st, b->d_probs,
                           b->d_red, j);
        RHQR_HIP(hipGetLastError());
        const int fg = fin_groups(j);
        hipLaunchKernelGGL(kb_fin, dim3(a * fg), dim3(1024), 0, st, b->d_probs, j, fg);
        RHQR_HIP(hipGetLastError());
      }
    }
  }
  hipLaunchKernelGGL((kb_finish<ST>), dim3(b->count, FINISH_CH), dim3(256), 0, st, b->d_probs);
  RHQR_HIP(hipGetLastError());
  return RHQR_OK;
}

int enqueue(rhqr_batch_s *b, hipStream_t st) {
  switch (b->dtype) {
    case RHQR_F64: return enqueue_typed<double>(b, st);
    case RHQR_F32: return enqueue_typed<float>(b, st);
    case RHQR_F16: return enqueue_typed<__half>(b, st);
    case RHQR_BF16: return enqueue_typed<__hip_bfloat16>(b, st);
  }
  return RHQR_ERR_UNSUPPORTED;
}

}  // namespace

extern "C" size_t rhqr_batch_workspace_size(const rhqr_problem *probs, int32_t count, int dtype) {
  if (check_problems(probs, count, dtype)) return 0;
  Layout L;
  if (plan(probs, count, dtype, &L)) return 0;
  return L.total;
}

extern "C" int rhqr_batch_create(const rhqr_problem *probs, int32_t count, int dtype, int opts,
                                 void *d_ws, size_t ws_bytes, void *stream, rhqr_batch_t *out) {
  int rc = check_problems(probs, count, dtype);
  if (rc) return rc;
  const int scaling = opts & 0xff;
  const int panel = (opts >> 8) & 0xff;
  const int outer = (opts >> 16) & 0xff;
  if ((scaling != RHQR_SCALE_UNIT_PIVOT && scaling != RHQR_SCALE_SQRT2) || panel == 1 ||
      panel > BATCH_MAXPB || ((unsigned)opts >> 24) != 0 ||
      (outer != 0 && (panel < 2 || outer <= panel || outer > BATCH_MAXPB || outer % panel != 0)))
    return -4;
  if (!d_ws) return -5;
  if (!out) return -8;
  Layout L;
  rc = plan(probs, count, dtype, &L);
  if (rc) return rc;
  if (ws_bytes < L.total) return RHQR_ERR_WORKSPACE;
  hipStream_t st = (hipStream_t)stream;
  char *ws = (char *)d_ws;
  const int tpw = batch_tpw(dtype);
  const size_t es = dtype_size(dtype);

  rhqr_batch_s *b = new rhqr_batch_s();
  b->dtype = dtype;
  b->kind = probs[0].sketch->kind;
  b->count = count;
  b->tpw = tpw;
  b->panel = panel;
  b->outer = outer;
  b->pan_start = L.pan_start;
  b->order = L.order;
  b->tall_start = L.tall_start;
  b->red_start = L.red_start;
  b->sk_blocks = L.sk_start[count];
  b->cols = L.col_start[count];
  std::vector<SketchJob> jobs(count);
  std::vector<BlockMap> tall_map(L.tall_start[count]), red_map(L.red_start[count]),
      sk_map(L.sk_start[count]), col_map(L.col_start[count]), pan_map(L.pan_start[count]);
  std::vector<ThinQBlock> qmap((size_t)L.qblocks_total);
  b->qjob.resize(count);
  b->qblocks = L.qblocks_total;
  b->qtiles_max = L.qtiles_max;
  int64_t qpos = 0;
  b->hp.resize(count);
  for (int s = 0; s < count; ++s) {
    const rhqr_problem &q = probs[L.order[s]];
    const rhqr_sketch_s *h = q.sketch;
    const int32_t m = h->m, Lr = h->l + h->m;
    b->ms.push_back(m);
    b->maxm = std::max(b->maxm, m);
    b->maxL = std::max(b->maxL, Lr);
    b->qa = std::max(b->qa, h->l <= SK_TPB ? 1 : h->l <= 2 * SK_TPB ? 2 : h->l <= 4 * SK_TPB ? 4 : 8);
    char *region = ws + L.off[s];
    const size_t lb = loop_ws_bytes(h->kind, dtype, h->n, m, h->l);
    LoopWs lw;
    rc = loop_ws_carve(region, lb, h->kind, dtype, h->n, m, h->l, &lw);
    if (rc) {
      delete b;
      return rc;
    }
    double *Z = (double *)(region + align_up(lb));
    double *skpart = (double *)(region + align_up(lb) + align_up(sizeof(double) * (size_t)Lr * m));
    int gt0;
    size_t skb0;
    sketch_tail_partials_size(h, m, &gt0, &skb0);
    double *Cc = (double *)((char *)skpart + align_up(skb0));
    double *Gc = (double *)((char *)Cc + align_up(sizeof(double) * (size_t)m * BATCH_MAXPB));
    double *Mq = (double *)((char *)Gc + align_up(sizeof(double) * (size_t)m * BATCH_MAXPB));
    b->mq.push_back(Mq);
    b->hs.push_back(h);
    b->skpart.push_back(skpart);
    b->skbytes.push_back(skb0);
    b->zs.push_back(Z);
    b->qmf.push_back((char *)Mq + align_up(sizeof(double) * (size_t)m * m));
    LoopArgs a;
    a.kind = h->kind;
    a.dtype = dtype;
    a.n = h->n;
    a.m = m;
    a.l = h->l;
    a.W = q.d_W;
    a.ldw = q.ldw;
    a.Z = Z;
    a.ldz = Lr;
    a.S = q.d_S;
    a.lds = q.lds;
    a.T = q.d_T;
    a.ldt = q.ldt;
    a.R = q.d_R;
    a.ldr = q.ldr;
    a.scaling = scaling;
    a.signs = h->d_signs;
    a.rows = h->d_rows;
    a.omega = h->d_omega;  // null for the SRHT
    a.defer = 1;
    b->hp[s] = make_col_problem(a, lw, tpw);
    b->hp[s].C = Cc;
    b->hp[s].G = Gc;
    SketchJob &jb = jobs[s];
    jb.X = q.d_W;
    jb.ldx = q.ldw;
    jb.n = h->n;
    jb.m = m;
    jb.l = h->l;
    jb.ngroups = L.ngroups[s];
    jb.gt = (int32_t)L.gt[s];
    jb.aligned = ((uintptr_t)q.d_W % 16 == 0) && ((q.ldw * (int64_t)es) % 16 == 0);
    jb.signs = h->d_signs;
    jb.rows = h->d_rows;
    jb.part = skpart;
    jb.Z = Z;
    jb.ldz = Lr;
    jb.scale = 1.0 / std::sqrt((double)h->l);
    for (int64_t k = 0; k < L.nparts[s]; ++k) tall_map[L.tall_start[s] + k] = {s, (int32_t)k};
    for (int64_t k = 0; k < L.gred[s]; ++k) red_map[L.red_start[s] + k] = {s, (int32_t)k};
    if (h->kind == RHQR_SKETCH_SRHT)  // the blocks of the one-launch SRHT pre-sketch
      for (int64_t k = 0; k < (int64_t)m * L.gt[s]; ++k) sk_map[L.sk_start[s] + k] = {s, (int32_t)k};
    for (int32_t k = 0; k < m; ++k) col_map[L.col_start[s] + k] = {s, k};
    for (int64_t k = 0; k < L.npanel[s]; ++k) pan_map[L.pan_start[s] + k] = {s, (int32_t)k};
    ThinQJob &qj = b->qjob[s];
    qj = ThinQJob{};
    qj.n = h->n;
    qj.ldu = q.ldw;
    qj.lds = q.lds;
    qj.ldt = q.ldt;
    qj.groups = L.qgroups[s];
    qj.m = m;
    qj.tiles = L.qtiles[s];
    qj.Kp = L.qkp[s];
    qj.U = q.d_W;
    qj.S = q.d_S;
    qj.T = q.d_T;
    qj.Mq = Mq;
    qj.qmf = b->qmf.back();
    for (int64_t k = 0; k < L.qblocks[s]; ++k) qmap[qpos++] = {s, (int32_t)k};
  }
  b->d_probs = (ColProblem *)(ws + L.off_probs);
  b->d_jobs = (SketchJob *)(ws + L.off_jobs);
  b->d_tall = (BlockMap *)(ws + L.off_tall);
  b->d_red = (BlockMap *)(ws + L.off_red);
  b->d_sk = (BlockMap *)(ws + L.off_sk);
  b->d_col = (BlockMap *)(ws + L.off_col);
  b->d_pan = (BlockMap *)(ws + L.off_pan);
  b->d_qjobs = (ThinQJob *)(ws + L.off_qjobs);
  b->d_qmap = (ThinQBlock *)(ws + L.off_qmap);
  auto up = [&](void *dst, const void *src, size_t bytes) -> int {
    if (bytes == 0) return RHQR_OK;
    RHQR_HIP(hipMemcpyAsync(dst, src, bytes, hipMemcpyHostToDevice, st));
    return RHQR_OK;
  };
  rc = up(b->d_probs, b->hp.data(), sizeof(ColProblem) * count);
  if (!rc) rc = up(b->d_jobs, jobs.data(), sizeof(SketchJob) * count);
  if (!rc) rc = up(b->d_tall, tall_map.data(), sizeof(BlockMap) * tall_map.size());
  if (!rc) rc = up(b->d_red, red_map.data(), sizeof(BlockMap) * red_map.size());
  if (!rc) rc = up(b->d_sk, sk_map.data(), sizeof(BlockMap) * sk_map.size());
  if (!rc) rc = up(b->d_col, col_map.data(), sizeof(BlockMap) * col_map.size());
  if (!rc) rc = up(b->d_pan, pan_map.data(), sizeof(BlockMap) * pan_map.size());
  if (!rc) rc = up(b->d_qmap, qmap.data(), sizeof(ThinQBlock) * qmap.size());
  if (!rc && hipStreamSynchronize(st) != hipSuccess) rc = RHQR_ERR_HIP;
  if (!rc && hipStreamCreateWithFlags(&b->cap, hipStreamNonBlocking) != hipSuccess) rc = RHQR_ERR_HIP;
  if (!rc && hipHostMalloc((void **)&b->h_qjobs, sizeof(ThinQJob) * count, hipHostMallocDefault) !=
                 hipSuccess)
    rc = RHQR_ERR_HIP;
  if (!rc && hipEventCreateWithFlags(&b->qev, hipEventDisableTiming) != hipSuccess)
    rc = RHQR_ERR_HIP;
  if (rc) {
    if (b->qev) (void)hipEventDestroy(b->qev);
    if (b->h_qjobs) (void)hipHostFree(b->h_qjobs);
    if (b->cap) (void)hipStreamDestroy(b->cap);
    delete b;
    return rc;
  }
  *out = b;
  return RHQR_OK;
}

extern "C" int rhqr_batch_factor(rhqr_batch_t b, int use_graph, void *stream) {
  if (!b) return -1;
  hipStream_t st = (hipStream_t)stream;
  if (!use_graph) return enqueue(b, st);
  if (!b->exec) {
    RHQR_HIP(hipStreamBeginCapture(b->cap, hipStreamCaptureModeThreadLocal));
    const int rc = enqueue(b, b->cap);
    hipGraph_t g = nullptr;
    const hipError_t ec = hipStreamEndCapture(b->cap, &g);
    if (rc) {
      if (g) (void)hipGraphDestroy(g);
      return rc;
    }
    RHQR_HIP(ec);
    b->graph = g;
    RHQR_HIP(hipGraphInstantiate(&b->exec, b->graph, nullptr, nullptr, 0));
  }
  RHQR_HIP(hipGraphLaunch(b->exec, st));
  return RHQR_OK;
}

extern "C" int rhqr_batch_thin_q(rhqr_batch_t b, void *const *d_Q, const int64_t *ldq,
                                 void *stream) {
  if (!b) return -1;
  if (!d_Q) return -2;
  if (!ldq) return -3;
  for (int s = 0; s < b->count; ++s) {
    const int i = b->order[s];
    if (d_Q[i] && ldq[i] < b->hp[s].n) return -3;
  }
  hipStream_t st = (hipStream_t)stream;
  // one launch per stage over every problem, unless a float64/float32
  // problem has columns that are not 16-byte aligned (then problem by problem)
  const size_t es = dtype_size(b->dtype);
  bool batched = true;
  for (int s = 0; s < b->count && es >= 4; ++s) {
    const int i = b->order[s];
    const ThinQJob &t = b->qjob[s];
    if (d_Q[i] && !((uintptr_t)t.U % 16 == 0 && (uintptr_t)d_Q[i] % 16 == 0 &&
                    (t.ldu * (int64_t)es) % 16 == 0 && (ldq[i] * (int64_t)es) % 16 == 0))
      batched = false;
  }
  if (batched) {
    if (b->qev_pending) RHQR_HIP(hipEventSynchronize(b->qev));  // the staging table is free
    for (int s = 0; s < b->count; ++s) {
      const int i = b->order[s];
      ThinQJob t = b->qjob[s];
      if (d_Q[i]) {
        t.Q = d_Q[i];
        t.ldq = ldq[i];
        const char *u1 = (const char *)t.U + (size_t)t.m * es;
        const char *q1 = (const char *)d_Q[i] + (size_t)t.m * es;
        t.aligned = ((uintptr_t)u1 % 16 == 0) && ((uintptr_t)q1 % 8 == 0) &&
                    ((t.ldu * (int64_t)es) % 16 == 0) && ((ldq[i] * (int64_t)es) % 8 == 0);
      } else {
        t.m = 0;  // skipped
        t.tiles = 0;
      }
      b->h_qjobs[s] = t;
    }
    RHQR_HIP(hipMemcpyAsync(b->d_qjobs, b->h_qjobs, sizeof(ThinQJob) * b->count,
                            hipMemcpyHostToDevice, st));
    RHQR_HIP(hipEventRecord(b->qev, st));
    b->qev_pending = true;
    return launch_thin_q_batched(b->dtype, b->count, b->maxm, b->qtiles_max, b->d_qjobs, b->d_qmap,
                                 b->qblocks, st);
  }
  for (int s = 0; s < b->count; ++s) {
    const int i = b->order[s];
    if (!d_Q[i]) continue;
    const ColProblem &P = b->hp[s];
    const int rc = launch_thin_q(b->dtype, P.n, P.m, P.W, P.ldw, P.S, P.lds, P.T, P.ldt, b->mq[s],
                                 b->qmf[s], d_Q[i], ldq[i], st);
    if (rc) return rc;
  }
  return RHQR_OK;
}

extern "C" int rhqr_batch_status(rhqr_batch_t b, void *stream, int32_t *h_info) {
  if (!b) return -1;
  if (!h_info) return -3;
  hipStream_t st = (hipStream_t)stream;
  std::vector<int32_t> w(2 * (size_t)b->count, 0);  // per problem: breakdown, non-finite
  for (int s = 0; s < b->count; ++s)
    RHQR_HIP(hipMemcpyAsync(&w[2 * (size_t)s], b->hp[s].status, 2 * sizeof(int32_t),
                            hipMemcpyDeviceToHost, st));
  RHQR_HIP(hipStreamSynchronize(st));
  for (int s = 0; s < b->count; ++s)
    h_info[b->order[s]] = w[2 * s + 1] ? -w[2 * s + 1] : w[2 * s];
  return RHQR_OK;
}

extern "C" int rhqr_batch_destroy(rhqr_batch_t b) {
  if (!b) return -1;
  if (b->exec) (void)hipGraphExecDestroy(b->exec);
  if (b->graph) (void)hipGraphDestroy(b->graph);
  if (b->cap) (void)hipStreamDestroy(b->cap);
  if (b->qev) (void)hipEventDestroy(b->qev);
  if (b->h_qjobs) (void)hipHostFree(b->h_qjobs);
  delete b;
  return RHQR_OK;
}
