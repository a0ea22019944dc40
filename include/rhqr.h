/*
 * rhqr.h -- C ABI of the MI355X (gfx950) randomized Householder QR library.
 *
 * Method: L. Grigori, E. Timsit, "Randomized Householder QR", arXiv 2405.10923.
 * The library factors a tall-skinny W (n x m, m << n) as
 *     W = (I_n - U T (Psi U)^t Psi) [R; 0] = Q R,      (Psi Q)^t (Psi Q) = I_m,
 * where Psi = [I_m 0; 0 Omega] (eq. psi, Sec. 3.1) keeps the first m rows and
 * sketches the remaining n-m rows with an l x (n-m) embedding Omega (Sec. 2.3).
 *
 * Conventions shared by every entry point
 *  - Matrices are column-major with an explicit leading dimension (ld >= rows).
 *  - Pointers named d_* are device pointers (HBM), pointers named h_* are host
 *    pointers.  The caller owns every input and output buffer; the library
 *    allocates device memory only inside the handles it creates (freed by the
 *    matching *_destroy) and never retains caller pointers after a call.
 *  - n-row data (W, U, Q, X) is stored in the element type `dtype`
 *    (RHQR_F64/F32/F16/BF16).  Sketch-space data (Psi X, S = Psi U, T, R, H)
 *    is always float64 -- the paper keeps the low-dimensional operations in
 *    high precision (Sec. 8, mixed-precision experiment).
 *  - Arithmetic on n-row data runs in float64 for RHQR_F64 and in float32 for
 *    the other types (FP32 accumulation).
 *  - Every call is asynchronous on `stream` (a hipStream_t, NULL = the null
 *    stream) unless stated otherwise; arguments are validated synchronously,
 *    before anything is launched.
 *  - Return value: RHQR_OK (0) on success; -i if argument i (1-based) is
 *    invalid; RHQR_ERR_HIP if a HIP call failed; RHQR_ERR_WORKSPACE if the
 *    workspace is too small.  Numerical breakdown is not an error return; it is
 *    reported through rhqr_status (below).
 */
#ifndef RHQR_H
#define RHQR_H

#include <stddef.h>
#include <stdint.h>

#ifndef RHQR_API
#define RHQR_API __attribute__((visibility("default")))
#endif

#ifdef __cplusplus
extern "C" {
#endif

enum {
  RHQR_OK = 0,
  RHQR_ERR_HIP = -1000,
  RHQR_ERR_WORKSPACE = -1001,
  RHQR_ERR_UNSUPPORTED = -1002
};

typedef enum { RHQR_F64 = 0, RHQR_F32 = 1, RHQR_F16 = 2, RHQR_BF16 = 3 } rhqr_dtype;

/* Sketch kinds (Sec. 2.3). */
typedef enum {
  RHQR_SKETCH_SRHT = 0,   /* Omega = sqrt(N/l) P H D on R^N, N = 2^ceil(log2 n) */
  RHQR_SKETCH_GAUSS = 1   /* Omega = G / sqrt(l), G iid N(0,1), stored densely  */
} rhqr_sketch_kind;

/* Reflector scaling of RHVector (Alg. 2, scaling line). */
typedef enum {
  RHQR_SCALE_UNIT_PIVOT = 0, /* u_jj = 1,  beta = |gamma| / rho  (LAPACK-like) */
  RHQR_SCALE_SQRT2 = 1       /* ||Psi u||^2 = 2,  beta = 1                     */
} rhqr_scaling;

/* recRHQR modes (Alg. 6 and its comparator of Sec. 8). */
typedef enum {
  RHQR_REC_M = 0,      /* U_2 = W_2 ut(T^t S^t Psi W)^-1, Q = [I;0] - U T U_1^t */
  RHQR_REC_RCHOL = 1   /* Q = W R^-1 (randomized Cholesky QR)                    */
} rhqr_rec_mode;

typedef struct rhqr_sketch_s *rhqr_sketch_t;
typedef struct rhqr_arnoldi_s *rhqr_arnoldi_t;

/* ------------------------------------------------------------------------
 * Sketch handle.  Draws Psi for problems with n rows and an m-row head.
 *   kind   : RHQR_SKETCH_SRHT or RHQR_SKETCH_GAUSS
 *   n, m, l: 0 <= m < n, 0 < l <= N (SRHT; l <= 4096) or l >= 1 (GAUSS);
 *            m = 0 gives Psi = Omega on every row (for rhqr_trim_factor; the
 *            entry points built on Psi = [I_m 0; 0 Omega] need m >= 1)
 *   seed   : Philox4x64-10 key word 0 (key word 1 selects the stream)
 *   d_omega: GAUSS only, optional caller-supplied l x (n-m) float64 Omega
 *            (ld_omega >= l); it is copied.  NULL: Omega is drawn on the
 *            device from the seed (Box-Muller, entries N(0, 1/l)).
 * The draw (random signs, the l sampled rows, or Omega) runs on the device,
 * on `stream`; the call synchronises `stream` before it returns.
 * Passage: Sec. 2.3 (Gaussian and SRHT embeddings), eq. psi.
 * ---------------------------------------------------------------------- */
RHQR_API int rhqr_sketch_create(int kind, int64_t n, int32_t m, int32_t l, uint64_t seed,
                       const double *d_omega, int64_t ld_omega, void *stream,
                       rhqr_sketch_t *out);
RHQR_API int rhqr_sketch_destroy(rhqr_sketch_t h);

/* Copies of the draw, for inspection: h_signs receives ceil(N/64) words (bit
 * i%64 of word i/64 set <=> D_ii = -1), h_rows the l sampled rows (int32,
 * increasing).  GAUSS: h_omega receives l x (n-m) entries (ld = l).  Any
 * pointer may be NULL.  Synchronous. */
RHQR_API int rhqr_sketch_get(rhqr_sketch_t h, uint64_t *h_signs, int32_t *h_rows, double *h_omega);
RHQR_API int rhqr_sketch_info(rhqr_sketch_t h, int64_t *n, int32_t *m, int32_t *l, int64_t *N, int32_t *kind);

/* ------------------------------------------------------------------------
 * rhqr_sketch: Y = Psi X  (RHSketch, Alg. 1).
 *   X  : n x k in dtype (ldx >= n), device;  Y: (l+m) x k float64 (ldy >= l+m)
 *   n must equal the handle's n.  ws: device workspace of at least
 *   rhqr_sketch_workspace_size(h, k) bytes.
 * SRHT order as Lemma srht: signs, Walsh-Hadamard transform, sampling; the
 * normalisation sqrt(N/l) * N^-1/2 = l^-1/2 is applied once to the samples.
 * ---------------------------------------------------------------------- */
RHQR_API size_t rhqr_sketch_workspace_size(rhqr_sketch_t h, int32_t k);
RHQR_API int rhqr_sketch(rhqr_sketch_t h, int dtype, int64_t n, int32_t k, const void *d_X,
                int64_t ldx, double *d_Y, int64_t ldy, void *d_ws, size_t ws_bytes,
                void *stream);

/* ------------------------------------------------------------------------
 * rhqr_factor: left-looking RHQR (Alg. 4) with RHVector (Alg. 2).
 *   d_W   : n x m in dtype, overwritten by U (unit lower-trapezoidal in the
 *           UNIT_PIVOT scaling).  The head m x m block of U is also in S.
 *   d_S   : (l+m) x m float64, S = Psi U
 *   d_T   : m x m float64, upper triangular; I - U T S^t Psi = P_1 ... P_m
 *   d_R   : m x m float64, upper triangular
 *   d_Q   : optional n x m thin Q factor in dtype (NULL to skip),
 *           Q = [I_m; 0] - U T U_1^t (Sec. 3.2)
 *   opts  : bits 0-7 rhqr_scaling; bits 8-15 panel width b (0 or 1: the
 *           column-by-column schedule of Alg. 4, every refresh reads all
 *           earlier reflectors; 2 <= b <= 32: before each panel of b columns
 *           the earlier reflectors are applied to the whole panel at once by a
 *           tall matrix product with C = T^t S^t Psi W_panel (the block form of
 *           Alg. 5 / Prop. 3.2), the columns inside a panel are refreshed as in
 *           Alg. 4 with the panel's own reflectors); bits 16-23 outer panel
 *           width B (0: one level; otherwise b >= 2, b < B <= 32 and B a
 *           multiple of b: the panels of b columns are grouped B at a time,
 *           each outer panel is updated from all earlier reflectors and each
 *           inner panel only from the reflectors of its outer panel).  Same
 *           factorization in exact arithmetic; the one synchronisation per
 *           column is kept.  Bits 24-27: transform tiles of 4096 rows per
 *           workgroup of the refresh + re-sketch pass, 0 (chosen from n), 1, 2
 *           or 4 (at least 2 for 2-byte storage): a tuning knob, the results
 *           differ only in the order of the transform's butterflies over the
 *           tile index and the summation order of the sketch partials.
 *           Bit 28: block RHQR exactly as Alg. 5 writes it, with blocks of b
 *           = bits 8-15 columns (1 <= b <= 32, outer width 0): before each
 *           block is factored (Alg. 4 over its columns, refresh coefficients
 *           from its own reflectors), every earlier block is applied to it in
 *           turn, each after a fresh sketch of the block.  Same factorization
 *           in exact arithmetic (U, S, T, R as without the bit).  For storage
 *           types narrower than float64 the block's head rows pass through
 *           the storage type between the earlier blocks' updates.
 *           Bit 29: right-looking RHQR as Alg. 3 writes it (bits 8-28 must
 *           then be 0): at step j the m - j trailing columns are sketched
 *           afresh, RHVector of column j is formed from the first of those
 *           sketches and the reflector is applied to every trailing column
 *           (W_{:,k} -= beta_j u_j s_j^t Psi w_k).  Same U, S, T, R as Alg. 4
 *           in exact arithmetic (T by Alg. 4's recursion); about three times
 *           the HBM traffic of the left-looking form.  For storage types
 *           narrower than float64 the trailing columns (head rows included)
 *           pass through the storage type after every step.
 *           Bits 30-31 must be 0.
 *   d_ws  : device workspace, >= rhqr_factor_workspace_size(h, dtype, m) bytes
 * One synchronisation per column: the refreshed column's sketch (Alg. 4).
 * Breakdown (rho_j = 0) gives an identity reflector (beta_j = 0, R_jj = 0) and
 * is reported by rhqr_status.
 * ---------------------------------------------------------------------- */
RHQR_API size_t rhqr_factor_workspace_size(rhqr_sketch_t h, int dtype, int32_t m);
RHQR_API int rhqr_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W, int64_t ldw,
                double *d_S, int64_t lds, double *d_T, int64_t ldt, double *d_R,
                int64_t ldr, void *d_Q, int64_t ldq, int opts, void *d_ws,
                size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * rhqr_factor_noalloc: rhqr_factor without a workspace argument, for callers
 * that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc).  Same arguments, results
 * and errors as rhqr_factor (bitwise the same outputs), minus d_ws/ws_bytes.
 * The workspace is a device array inside the library of
 * RHQR_NOALLOC_SCRATCH_BYTES (64 MiB) that every GPU the library runs on
 * holds until the process ends; the call allocates nothing.  Returns
 * RHQR_ERR_WORKSPACE when rhqr_factor_workspace_size(h, dtype, m) exceeds
 * that size (nothing is launched).  Every call on one GPU shares that GPU's
 * array: calls that overlap in time on one GPU (several streams or host
 * threads) race and must be serialised by the caller.
 *   d_info: optional (NULL to skip) device array of 2 int32 receiving, at the
 *           end of the call on `stream`, the first column (1-based) with
 *           rho_j = 0 and the first non-finite column, 0 if none (what
 *           rhqr_status reports for rhqr_factor).
 * ---------------------------------------------------------------------- */
#define RHQR_NOALLOC_SCRATCH_BYTES ((size_t)64 << 20)
RHQR_API int rhqr_factor_noalloc(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W,
                                 int64_t ldw, double *d_S, int64_t lds, double *d_T, int64_t ldt,
                                 double *d_R, int64_t ldr, void *d_Q, int64_t ldq, int opts,
                                 int32_t *d_info, void *stream);

/* Status of the last rhqr_factor / recrhqr_factor call that used this
 * workspace, in *h_info (host):
 *    0  every reflector was formed;
 *    j  (> 0) column j (1-based) was the first with rho_j = 0 (breakdown: the
 *       column is already eliminated, the reflector is the identity);
 *   -j  column j was the first whose rho_j or pivot entry y_j is NaN or
 *       infinite (a non-finite input, or overflow); this takes precedence over
 *       a breakdown, and every output from column j on is meaningless.
 * Returns -1 for d_ws NULL, -3 for h_info NULL.  Synchronises `stream`. */
RHQR_API int rhqr_status(const void *d_ws, void *stream, int32_t *h_info);

/* ------------------------------------------------------------------------
 * rhqr_rgs_factor: BLAS2-RGS (Alg. 9, Sec. 6), randomized Gram-Schmidt
 * obtained as left-looking RHQR of [0_{m x m}; W] with Psi = [I_m 0; 0 Omega]
 * and Omega applied to the n rows of W.  The head of every refreshed column
 * below its pivot is exactly zero, so the pivot sign is never flipped and
 * the Householder vectors are [e_j; q_j].
 *   h     : sketch handle with n + m rows and head m (its Omega acts on W)
 *   d_W   : n x m in dtype (ldw >= n), read only
 *   d_Q   : (n+m) x m in dtype (ldq >= n + m): rows m .. n+m-1 receive Q
 *           (Omega Q orthonormal, W = Q R), rows 0 .. m-1 receive I_m
 *   d_S   : (l+m) x m float64: [I_m; Omega Q]
 *   d_T   : m x m float64, unit upper triangular (I_m in exact arithmetic)
 *   d_R   : m x m float64, upper triangular with diagonal rho_j > 0
 *   opts  : the schedule bits of rhqr_factor (scaling must be UNIT_PIVOT)
 *   d_ws  : rhqr_rgs_workspace_size(h, dtype, m) bytes
 * Alg. 9's optional last line (Q <- Q T) is not applied.  Breakdown and
 * non-finite columns are reported by rhqr_status as for rhqr_factor.
 * ---------------------------------------------------------------------- */
RHQR_API size_t rhqr_rgs_workspace_size(rhqr_sketch_t h, int dtype, int32_t m);
RHQR_API int rhqr_rgs_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, const void *d_W,
                             int64_t ldw, void *d_Q, int64_t ldq, double *d_S, int64_t lds,
                             double *d_T, int64_t ldt, double *d_R, int64_t ldr, int opts,
                             void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * rhqr_trim_factor: left-looking trimRHQR (Alg. 12, Sec. 7) with
 * trimRHVector (Alg. 10): reflectors H_j = I - beta u (Omega u)^t
 * [0 Omega_{j:n}] that sketch only the rows from their pivot on, with an
 * Omega (l x n) over every row, so l may be smaller than m.
 *   h     : SRHT sketch handle with head 0 (rhqr_sketch_create(..., n, 0, l,
 *           ...)): its Omega acts on all n rows; its columns have unit norm,
 *           which the elimination needs (the Gaussian sketch's do not)
 *   dtype : RHQR_F64 or RHQR_F32 (n-row arithmetic in that type)
 *   d_W   : n x m, overwritten by U (u_j zero above row j; unit pivot in the
 *           UNIT_PIVOT scaling), 1 <= m <= min(n, 1024)
 *   d_S   : l x m float64 (lds = l), S = Omega U
 *   d_T   : m x m float64: H_1 ... H_m = I - U T ut((Omega U)^t Omega)
 *   d_Tt  : m x m float64 (T~): H_m ... H_1 = I - U T~^t ut((Omega U)^t Omega)
 *   d_R   : m x m float64 upper triangular: W = H_1 ... H_m [R; 0]
 *   d_Q   : optional n x m thin factor Q = H_1 ... H_m [I_m; 0] in dtype
 *   opts  : bits 0-7 rhqr_scaling (alpha = 1/v_j, or sqrt 2 / ||Omega v||)
 *   d_ws  : rhqr_trim_workspace_size(h, dtype, m) bytes
 * One synchronisation per column (the sketch of the refreshed column).
 * Breakdown and non-finite columns are reported by rhqr_status(d_ws).
 * ---------------------------------------------------------------------- */
RHQR_API size_t rhqr_trim_workspace_size(rhqr_sketch_t h, int dtype, int32_t m);
RHQR_API int rhqr_trim_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, void *d_W,
                              int64_t ldw, double *d_S, int64_t lds, double *d_T, int64_t ldt,
                              double *d_Tt, int64_t ldtt, double *d_R, int64_t ldr, void *d_Q,
                              int64_t ldq, int opts, void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * Column scaling for low-precision storage (the mixed-precision experiment of
 * Sec. 8, where W is held in half precision): before W is rounded to a
 * narrow type its columns are scaled to unit max-norm, and R is scaled back
 * afterwards, so that W = Q (R D) for the unscaled W.
 *   rhqr_colscale: d_scale[j] = max_i |W_ij| (1 for a zero column), computed
 *     in float64; d_Wout = W D^-1 rounded to dtype (to float32 first, then to
 *     the 2-byte type, both round-to-nearest-even).  d_W64: n x m float64
 *     (ldw >= n), read only; d_Wout: n x m in dtype (ldo >= n), may not
 *     overlap d_W64; d_scale: m float64.  Device pointers; asynchronous.
 *   rhqr_scale_r: R <- R D, column j of the m x m upper-triangular R (ldr >=
 *     m) multiplied by d_scale[j].  Device pointers; asynchronous.
 * ---------------------------------------------------------------------- */
RHQR_API int rhqr_colscale(int dtype, int64_t n, int32_t m, const double *d_W64, int64_t ldw,
                           void *d_Wout, int64_t ldo, double *d_scale, void *stream);
RHQR_API int rhqr_scale_r(int32_t m, double *d_R, int64_t ldr, const double *d_scale,
                          void *stream);

/* ------------------------------------------------------------------------
 * recrhqr_factor: recRHQR (Alg. 6), one synchronisation.
 *   Z = Psi W; Householder QR of Z on the device in float64 gives S, T, R;
 *   mode RHQR_REC_M: U_2 solves W_2 = U_2 ut(T^t S^t Z) (row-wise forward
 *   substitution), U_1 = S_{1:m}; Q (optional) = [I;0] - U T U_1^t.
 *   mode RHQR_REC_RCHOL: Q = W R^-1 (d_U may be NULL).
 *   d_W is read only; d_U (n x m, dtype) receives U; d_Q optional.
 * ---------------------------------------------------------------------- */
RHQR_API size_t recrhqr_workspace_size(rhqr_sketch_t h, int dtype, int32_t m);
RHQR_API int recrhqr_factor(rhqr_sketch_t h, int dtype, int64_t n, int32_t m, const void *d_W,
                   int64_t ldw, void *d_U, int64_t ldu, double *d_S, int64_t lds,
                   double *d_T, int64_t ldt, double *d_R, int64_t ldr, void *d_Q,
                   int64_t ldq, int mode, void *d_ws, size_t ws_bytes, void *stream);

/* ------------------------------------------------------------------------
 * RHQR-Arnoldi (Alg. 7, Sec. 5).  The operator stays with the caller.
 *   rhqr_arnoldi_create: state for up to mmax Arnoldi steps; the sketch handle
 *     must have head m = mmax + 1 (the loop forms mmax + 1 reflectors).  The
 *     state owns its device memory (basis U, n x (mmax+1) in dtype, S, T, H,
 *     and the n-vectors of the GMRES driver below).
 *   rhqr_arnoldi_start(r0): r0 = b - A x0 (n, dtype, device).  Forms u_1 from
 *     r0 and its sketch, writes q_1 (n, dtype, device) and, on the host,
 *     beta = (h_0)_1 = -sigma_1 rho_1 so that r0 = beta q_1.  Synchronous.
 *   rhqr_arnoldi_step(w): w = A q_j (n, dtype, device) for the current j.
 *     Sketches w, refreshes it with the j reflectors (w - U T^t S^t Psi w),
 *     re-sketches, forms u_{j+1}, writes h_j ((mmax+1) float64, device; rows
 *     > j+1 are zero) and q_{j+1} (n, dtype, device; NULL to skip).  Returns
 *     -1 once mmax steps have been taken.
 *   rhqr_arnoldi_solution(j, y): x += Q_j y (y: j float64 values, device;
 *     x: n, dtype, device), 1 <= j <= number of steps taken.
 *   rhqr_arnoldi_basis: device pointers of U (tail rows; the head rows of the
 *     Householder vectors are the head rows of S), S ((l+mmax+1) x (mmax+1),
 *     ld l+mmax+1) and T ((mmax+1) x (mmax+1), ld mmax+1).  The most recent
 *     column of U is stored before its division by alpha.
 *   rhqr_arnoldi_solve_ls(j, y, res): the small least-squares problem of
 *     Alg. 8 and of the proposition after it, min_y ||beta e_1 - H y||_2 with
 *     H the (j+1) x j upper Hessenberg matrix [h_1 .. h_j] of the steps taken
 *     and beta = (h_0)_1 = -sigma_1 rho_1 from rhqr_arnoldi_start, solved on
 *     the device in float64 by Givens rotations and back substitution.
 *     d_y: j float64 (device) receives y; d_res: optional (NULL to skip) one
 *     float64 (device) receiving the minimal residual |(Q^t beta e_1)_{j+1}|,
 *     which equals ||Psi (r_0 - A Q_j y)|| (the sketched GMRES residual).
 *     1 <= j <= number of steps taken (-2 otherwise).  Asynchronous.
 *   rhqr_gmres_csr: restarted RHQR-GMRES(mmax) (Alg. 8) on a CSR operator,
 *     run entirely by the library on the handle's basis and vectors: per
 *     cycle r = b - A x in float64 (rounded to dtype for the basis), the
 *     Arnoldi process of mmax steps (Alg. 7), rhqr_arnoldi_solve_ls, and
 *     x += Q y accumulated in float64; the true relative residual
 *     ||b - A x|| / ||b|| is recomputed in float64 after every cycle and the
 *     iteration stops once it is <= tol or after max_cycles cycles.
 *     d_ptr, d_idx, d_val: the CSR operator as for rhqr_spmv_csr (n = the
 *     handle's n); d_b: n float64; d_x: n float64, x_0 on entry, the solution
 *     on return.  h_hist: optional host array of max_cycles doubles receiving
 *     the relative residual after each cycle; h_cycles, h_steps: optional
 *     host outputs (cycles run, Arnoldi steps taken).  Synchronises `stream`
 *     once per cycle (the convergence test).  Returns -7 for tol < 0 or NaN,
 *     -8 for max_cycles < 1.
 * rhqr_spmv_csr: y = A x for A in CSR (row pointers int64, column indices
 *   int32, values float64; n rows), x and y in dtype, float64 accumulation.
 *   Device pointers; asynchronous.
 * ---------------------------------------------------------------------- */
RHQR_API int rhqr_arnoldi_create(rhqr_sketch_t h, int dtype, int64_t n, int32_t mmax, void *stream,
                        rhqr_arnoldi_t *out);
RHQR_API int rhqr_arnoldi_destroy(rhqr_arnoldi_t a);
RHQR_API int rhqr_arnoldi_start(rhqr_arnoldi_t a, const void *d_r0, void *d_q1, double *h_beta,
                       void *stream);
RHQR_API int rhqr_arnoldi_step(rhqr_arnoldi_t a, const void *d_w, void *d_qnext, double *d_hcol,
                      void *stream);
RHQR_API int rhqr_arnoldi_solution(rhqr_arnoldi_t a, int32_t j, const double *d_y, void *d_x,
                          void *stream);
RHQR_API int rhqr_arnoldi_basis(rhqr_arnoldi_t a, void **d_U, double **d_S, double **d_T);
RHQR_API int rhqr_arnoldi_solve_ls(rhqr_arnoldi_t a, int32_t j, double *d_y, double *d_res,
                                   void *stream);
RHQR_API int rhqr_gmres_csr(rhqr_arnoldi_t a, const int64_t *d_ptr, const int32_t *d_idx,
                            const double *d_val, const double *d_b, double *d_x, double tol,
                            int32_t max_cycles, double *h_hist, int32_t *h_cycles,
                            int64_t *h_steps, void *stream);
RHQR_API int rhqr_spmv_csr(int dtype, int64_t n, const int64_t *d_ptr, const int32_t *d_idx,
                  const double *d_val, const void *d_x, void *d_y, void *stream);

/* ------------------------------------------------------------------------
 * Batched left-looking RHQR: `count` independent factorizations (Alg. 4 with
 * RHVector, Alg. 2), each with its own n, m, l (taken from its sketch
 * handle), W, S, T and R as in rhqr_factor, all in one element type and one
 * sketch kind (every handle SRHT, or every handle Gaussian).
 *   rhqr_problem: sketch (handle with the problem's n, head m and l),
 *     d_W (n x m in dtype, ld >= n; overwritten by U), d_S ((l+m) x m float64),
 *     d_T, d_R (m x m float64).  Device pointers, owned by the caller.
 *   rhqr_batch_workspace_size: device workspace bytes for the batch (0 if a
 *     problem is invalid).
 *   rhqr_batch_create: validates the problems (m <= 1024, l <= 4096, leading
 *     dimensions, one sketch kind), lays the descriptors and per-problem scratch out in the
 *     caller's workspace d_ws (kept by the batch until rhqr_batch_destroy: the
 *     caller must keep it alive), uploads them on `stream` and synchronises.
 *     opts: bits 0-7 rhqr_scaling; bits 8-15 panel width b and bits 16-23
 *     outer panel width B with rhqr_factor's meaning and rules (b = 0: column
 *     schedule; 2 <= b <= 32: blocked, one level when B = 0, else outer
 *     panels of B, a multiple of b, b < B <= 32); other bits 0.
 *     Returns -1 for an invalid problem array, -3 bad dtype, -4 bad opts,
 *     -5 null workspace, RHQR_ERR_WORKSPACE if ws_bytes is too small.
 *   rhqr_batch_factor: factors every problem of the batch.  The work is a
 *     fixed sequence of kernel launches (no allocation, no host
 *     synchronisation, no memset): the pre-sketch (one launch over every
 *     problem for SRHT batches; per problem, as rhqr_sketch, for Gaussian
 *     ones), then per column index j one refresh + re-sketch launch, one
 *     reduction and one float64 step over the problems with m_p > j.  use_graph != 0: the sequence is captured once into a hipGraph
 *     (on the batch's own stream) and the graph is launched on `stream`; later
 *     calls replay it.  Each problem's U, S, T, R equal those of rhqr_factor
 *     with the same schedule bitwise (same device code, same choice of
 *     matrix cores or vector units per panel, same reduction orders), given
 *     the batch's transform tiles per workgroup (1; 2 for 2-byte storage:
 *     rhqr_factor's own choice below 2^21 rows, else opts bits 24-27).
 *   rhqr_batch_thin_q: after rhqr_batch_factor (on the same stream), the
 *     thin Q of every problem i with d_Q[i] != NULL: Q_i = [I_m; 0] -
 *     U_i T_i U_{i,1}^t (Sec. 3.2), n_i x m_i in the batch dtype, column-major
 *     with leading dimension ldq[i] >= n_i.  d_Q and ldq are host arrays of
 *     `count` entries in caller order (device pointers in d_Q, owned by the
 *     caller).  The same device code per entry and per workgroup as
 *     rhqr_factor's thin Q, so each Q_i equals the one rhqr_factor forms for
 *     that problem bitwise.  One launch per stage over all problems (a job
 *     table of the Q pointers is uploaded on `stream` from pinned memory the
 *     batch owns); problem by problem instead when a float64/float32 problem's
 *     U or Q columns are not 16-byte aligned.  Not part of the factorization
 *     graph.  Calls on one batch must be ordered (one stream): they share the
 *     batch's scratch.  Returns -1 for a null batch, -2 for a null d_Q, -3
 *     for a null ldq or ldq[i] < n_i (before any launch).
 *   rhqr_batch_status: h_info[i] (host, count entries, caller order) = the
 *     status of problem i as rhqr_status reports it (0; j > 0 for the first
 *     column with rho_j = 0; -j for the first non-finite column).
 *     Synchronous.
 * Not in the paper as such: the paper factors one matrix at a time; the batch
 * applies Alg. 4 to each problem independently.
 * ---------------------------------------------------------------------- */
typedef struct rhqr_problem {
  rhqr_sketch_t sketch;
  void *d_W;
  int64_t ldw;
  double *d_S;
  int64_t lds;
  double *d_T;
  int64_t ldt;
  double *d_R;
  int64_t ldr;
} rhqr_problem;
typedef struct rhqr_batch_s *rhqr_batch_t;

RHQR_API size_t rhqr_batch_workspace_size(const rhqr_problem *probs, int32_t count, int dtype);
RHQR_API int rhqr_batch_create(const rhqr_problem *probs, int32_t count, int dtype, int opts,
                               void *d_ws, size_t ws_bytes, void *stream, rhqr_batch_t *out);
RHQR_API int rhqr_batch_factor(rhqr_batch_t b, int use_graph, void *stream);
RHQR_API int rhqr_batch_thin_q(rhqr_batch_t b, void *const *d_Q, const int64_t *ldq,
                               void *stream);
RHQR_API int rhqr_batch_status(rhqr_batch_t b, void *stream, int32_t *h_info);
RHQR_API int rhqr_batch_destroy(rhqr_batch_t b);

/* ------------------------------------------------------------------------
 * Measurement aid (not part of the method).  Between rhqr_profile_begin() and
 * rhqr_profile_end(), every launch of the kernels listed below records a start
 * and an end HIP event from its own dispatch, so each duration is that
 * kernel's own (launch gaps excluded).  Classes:
 *   RHQR_PROF_TALL        per-column refresh + re-sketch pass (Alg. 4)
 *   RHQR_PROF_PANEL_MX    panel update of the blocked schedule, matrix cores
 *   RHQR_PROF_PANEL_VALU  panel update of the blocked schedule, vector units
 *   RHQR_PROF_PRESKETCH   multi-column sketch Psi X (Alg. 1): the SRHT tile
 *                         pass or the Gaussian product, without its finish
 *   RHQR_PROF_RED         per-column reduction of the sketch partials
 *   RHQR_PROF_FIN         per-column float64 step (RHVector, T, c)
 *   RHQR_PROF_QTAIL       tail product of the thin Q (Sec. 3.2)
 *   RHQR_PROF_TRSM        blocked substitution of recRHQR (Alg. 6)
 *   RHQR_PROF_HQR         sketch-space Householder QR of recRHQR (Alg. 6)
 *   RHQR_PROF_RIGHT_VEC   per-column RHVector step of right-looking RHQR
 *                         (Alg. 3): s_j, R, T and the trailing coefficients
 *   RHQR_PROF_RIGHT_APPLY per-column row pass of right-looking RHQR (Alg. 3):
 *                         u_j stored, the trailing columns updated
 * rhqr_profile_end(nclass, h_ms, h_launches) synchronises the recorded events
 * and writes, for classes 0 .. nclass-1, the summed kernel time in ms
 * (h_ms[c]) and the number of launches (h_launches[c]); host arrays of nclass
 * entries, nclass <= RHQR_PROF_NCLASS (0: only close the window).  Returns -1
 * for a bad nclass, -2 / -3 for a NULL array, RHQR_ERR_HIP if an event
 * failed.  The window is process-wide and mutex-guarded: launches from every
 * host thread are collected.  Profiling adds two events per launch; time
 * work outside the window.
 * ---------------------------------------------------------------------- */
enum {
  RHQR_PROF_TALL = 0,
  RHQR_PROF_PANEL_MX = 1,
  RHQR_PROF_PANEL_VALU = 2,
  RHQR_PROF_PRESKETCH = 3,
  RHQR_PROF_RED = 4,
  RHQR_PROF_FIN = 5,
  RHQR_PROF_QTAIL = 6,
  RHQR_PROF_TRSM = 7,
  RHQR_PROF_HQR = 8,
  RHQR_PROF_RIGHT_VEC = 9,
  RHQR_PROF_RIGHT_APPLY = 10,
  RHQR_PROF_NCLASS = 11
};
RHQR_API int rhqr_profile_begin(void);
RHQR_API int rhqr_profile_end(int32_t nclass, double *h_ms, int64_t *h_launches);

#ifdef __cplusplus
}
#endif
#endif /* RHQR_H */
