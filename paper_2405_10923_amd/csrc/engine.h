// Column-loop engine of left-looking RHQR (Alg. 4) shared by rhqr_factor,
// recrhqr_factor (its sketch-space Householder QR runs the same loop with
// Psi = I) and the batched entry point.
#pragma once
#include "common.h"

struct LoopWs {
  int32_t *status;   // first column with rho_j = 0 (1-based), 0 if none
  double *dcpart;    // [m / 16] per-workgroup sums of d_p c_p (deferred last coefficient)
  double *fs;        // beta_j and e_j of the deferred last coefficient
  double *y;         // (l+m) sketch of the refreshed column
  double *sq;        // per-workgroup partial sums of squares
  double *dpart;     // [G_red][m] partial S^t y (masked to rows >= j)
  double *epart;     // [G_red][m] partial S^t z_{j+1}
  double *ypart;     // [G_red] partial y^t z_{j+1}
  double *scal;      // [m][4]: sigma, rho, alpha, beta
  double *c;         // c_{j+1} = T_j^t S_j^t z_{j+1}
  double *cf;        // c with the pending 1/alpha of the raw column folded in
  double *ia;        // [m] 1/alpha_j applied when u_j is stored
  double *Tt;        // m x m transpose of T (ld m)
  double *part;      // [ntiles][l] per-tile sketch partials
  void *skws;        // workspace of the multi-column pre-sketch
  size_t skws_bytes;
};

struct LoopArgs {
  int kind;           // RHQR_SKETCH_SRHT / GAUSS / IDENT
  int dtype;
  int64_t n;
  int32_t m, l;
  void *W;
  int64_t ldw;
  const double *Z;    // (l+m) x m pre-sketch (may alias W for IDENT)
  int64_t ldz;
  double *S;
  int64_t lds;
  double *T;
  int64_t ldt;
  double *R;
  int64_t ldr;
  int scaling;
  const uint64_t *signs;
  const int32_t *rows;
  const double *omega;  // l x (n-m), ld l
  int defer;          // the step of column j-1 left c_{j-1} to be finished by column j
  int tpw = 0;        // transform tiles per tall workgroup (0: chosen from n)
  int32_t c0 = 0;     // first reflector of the refresh coefficients (block RHQR, Alg. 5)
};

// Everything the per-column kernels read about one problem: its data, its
// sketch and its slice of the loop workspace.  Passed by value to the
// single-problem kernels; the batched kernels read an array of them from
// device memory.
struct ColProblem {
  void *W;
  int64_t ldw, n;
  int32_t m, l;
  const double *Z;
  int64_t ldz;
  double *S;
  int64_t lds;
  double *T;
  int64_t ldt;
  double *R;
  int64_t ldr;
  const uint64_t *signs;
  const int32_t *rows;
  const double *omega;
  double scale;        // l^-1/2 for the SRHT tile partials, 1 otherwise
  int64_t nparts;      // tall workgroups (= partial sketches per column)
  int32_t gred;        // reduction workgroups
  int32_t scaling, defer, aligned;
  int32_t c0 = 0;      // c_p = sum_{c0 <= q <= p} T_{q,p} (S^t z)_q: only the reflectors
                       // from c0 on (block RHQR, Alg. 5, refreshes inside one block)
  double *part, *y, *sq, *dpart, *epart, *ypart, *scal, *c, *cf, *ia, *Tt, *dcpart, *fs;
  int32_t *status;
  double *C, *G;       // panel coefficients of the blocked schedule (batched path)
};

// descriptor of (a, w) for tall workgroups of tpw transform tiles
ColProblem make_col_problem(const LoopArgs &a, const LoopWs &w, int tpw);

size_t loop_ws_bytes(int kind, int dtype, int64_t n, int32_t m, int32_t l);
int loop_ws_carve(void *ws, size_t bytes, int kind, int dtype, int64_t n, int32_t m, int32_t l,
                  LoopWs *out);
int run_column_loop(const LoopArgs &a, const LoopWs &w, hipStream_t st);
// single-column pieces of the loop (used by the Arnoldi process):
// the tall refresh + re-sketch pass of column j (j >= 1), and the float64 step
// (reduction, RHVector, T column; c_{j+1} when next != 0, from Z_{:, j+1}).
int engine_tall(const LoopArgs &a, const LoopWs &w, int32_t j, hipStream_t st);
int engine_step(const LoopArgs &a, const LoopWs &w, int32_t j, int next, hipStream_t st);
// blocked schedule: panels of `panel` (<= 32) columns, optionally grouped in
// outer panels of `outer` (a multiple of panel, <= 32; outer <= panel: one
// level); C and G are float64 scratch of m x 32 entries each
int run_column_loop_blocked(const LoopArgs &a, const LoopWs &w, int panel, int outer, double *C,
                            double *G, hipStream_t st);
// block RHQR as Alg. 5 writes it: blocks of b (<= 32) columns, each earlier
// block applied after a fresh sketch of the current block; C: m x 32 and G:
// 32 x 32 float64 scratch, Z: (l+m) x m float64 (the fresh sketches), skws:
// the multi-column sketch workspace for b columns
int run_column_loop_alg5(const rhqr_sketch_s *h, const LoopArgs &a, const LoopWs &w, int b,
                         double *C, double *G, double *Z, void *skws, size_t skws_bytes,
                         hipStream_t st);
// right-looking RHQR as Alg. 3 writes it: at step j the m - j trailing
// columns are sketched into Z ((l+m) x m float64) with the multi-column sketch
// workspace skws, then RHVector and the trailing update (right.hip)
int run_column_loop_right(const rhqr_sketch_s *h, const LoopArgs &a, const LoopWs &w, double *Z,
                          void *skws, size_t skws_bytes, hipStream_t st);
// thin Q = [I; 0] - U T U_1^t (Sec. 3.2); Mq: m x m float64 scratch, qmf:
// thin_q_bytes(m) bytes of scratch (2-byte storage: split coefficients)
size_t thin_q_bytes(int32_t m);
int launch_thin_q(int dtype, int64_t n, int32_t m, const void *U, int64_t ldu, const double *S,
                  int64_t lds, const double *T, int64_t ldt, double *Mq, void *qmf, void *Q,
                  int64_t ldq, hipStream_t st);
// The thin Q of many problems, one launch per stage over all of them (the
// same per-entry and per-workgroup code as launch_thin_q, so each Q is the
// single-problem one bitwise).  A job with m = 0 and tiles = 0 is skipped.
// float64/float32 need every job's U and Q 16-byte aligned (the matrix-core
// tail product); 2-byte storage takes any alignment.  Mq: m x m float64
// scratch, qmf: thin_q_bytes(m) bytes of scratch, per job.
struct ThinQJob {
  int64_t n, ldu, lds, ldt, ldq, groups;
  int32_t m, tiles, Kp, aligned;
  const void *U;
  const double *S, *T;
  double *Mq;
  void *qmf, *Q;
};
struct ThinQBlock {
  int32_t p, local;  // job, workgroup of its tail product
};
// workgroups of one problem's tail product and its geometry (tiles of Q's
// columns, row groups, padded coefficient rows)
int64_t thin_q_tail_blocks(int dtype, int64_t n, int32_t m, int32_t *tiles, int64_t *groups,
                           int32_t *Kp);
int launch_thin_q_batched(int dtype, int32_t count, int32_t maxm, int32_t maxtiles,
                          const ThinQJob *d_jobs, const ThinQBlock *d_map, int64_t nblocks,
                          hipStream_t st);
int launch_fill(void *p, size_t bytes, hipStream_t st);
// X M = B for `rows` rows (B, X n-row data in dtype, column-major; M upper
// triangular m x m float64): blocked forward substitution (recRHQR, Alg. 6).
// coef: trsm_coef_bytes(m) bytes of scratch; stage: trsm_stage_bytes(...)
// bytes (a float32 copy of X, 2-byte types only; may be NULL otherwise).
size_t trsm_coef_bytes(int32_t m);
size_t trsm_stage_bytes(int dtype, int64_t rows, int32_t m);
int launch_trsm_blocked(int dtype, const void *B, int64_t ldb, int64_t rows, int32_t m,
                        const double *M, int64_t ldm, void *X, int64_t ldx, double *coef,
                        float *stage, hipStream_t st);

constexpr int RED_CHUNK = 64;  // outputs per reduction workgroup
