/*
 * tsgmres.h -- C ABI of the MI355X (gfx950) library for s-step GMRES with
 * two-stage block orthogonalization.
 *
 * Method: I. Yamazaki, A. J. Higgins, E. G. Boman, D. B. Szyld, "Two-Stage Block
 * Orthogonalization to Improve Performance of s-step GMRES", arXiv:2402.15033.
 *
 * Conventions for every entry point
 *   - Pointers are DEVICE pointers (hipMalloc'd or torch CUDA/HIP tensors) unless
 *     the comment says "host".
 *   - Dense blocks are column-major with an explicit leading dimension.
 *   - Sparse matrices are CSR with int32 row pointers / column indices and float64
 *     values; row r holds entries row_ptr[r] .. row_ptr[r+1]-1.
 *   - `stream` is a hipStream_t passed as void* (NULL = the legacy default stream).
 *     All device work is enqueued on it, in order.
 *   - The caller owns every buffer it passes.  The library never frees caller
 *     memory; all O(n) scratch lives in a caller-provided workspace whose size is
 *     returned by the matching *_workspace_bytes() query.
 *   - Errors: no exception or abort crosses this ABI.  A negative status is a
 *     caller or runtime error detected before (or instead of) numerical work; a
 *     positive status is a numerical outcome.  tsg_last_error() returns a
 *     thread-local message describing the last non-OK status.
 */
#ifndef TSGMRES_H
#define TSGMRES_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  TSG_OK = 0,
  TSG_NOT_CONVERGED = 1,    /* max_iters reached; x holds the last iterate            */
  TSG_BREAKDOWN = 2,        /* a restart cycle could keep no basis vector              */
  TSG_ERR_INVALID_ARG = -1, /* bad sizes / NULL pointers / unsupported combination    */
  TSG_ERR_HIP = -2,         /* a HIP runtime call failed (message in tsg_last_error)  */
  TSG_ERR_WORKSPACE = -3,   /* workspace too small or misaligned (256-byte alignment) */
  TSG_ERR_UNSUPPORTED = -4  /* valid request outside what the library implements     */
} tsg_status;

/* Block orthogonalization scheme used inside a restart cycle.
 *   TWO_STAGE      Sec. V, Fig. 5 with s_hat = m: one BCGS-PIP per s-column panel
 *                  (stage 1), one CholQR of the m+1 columns at the end of the cycle
 *                  (stage 2).  One global reduction per panel plus one per cycle.
 *                  A panel whose Pythagorean Gram fails the pivot test (beyond the
 *                  PIP stability limit of Sec. IV-C) is projected explicitly and
 *                  orthogonalized by a second PIP pass (one more reduction).
 *   BCGS_PIP2      Sec. IV-C, Fig. 4b (two reductions per panel).
 *   BCGS2_CHOLQR2  Sec. IV-B, Fig. 2b with CholQR2 then CholQR (five per panel).
 *   CGS2           standard GMRES(m), classical Gram-Schmidt twice, one vector per
 *                  iteration (the paper's "standard GMRES" baseline, Tables 2-4). */
typedef enum {
  TSG_ORTHO_TWO_STAGE = 0,
  TSG_ORTHO_BCGS_PIP2 = 1,
  TSG_ORTHO_BCGS2_CHOLQR2 = 2,
  TSG_ORTHO_CGS2 = 3
} tsg_ortho;

/* s-step basis w_i = (A w_{i-1} - theta_i w_{i-1} + tau_i w_{i-2}) / sigma_i
 * (matrix-powers kernel, Sec. III; tau = 0 except in LEJA).  [lo, hi] is the Gershgorin
 * interval computed at tsg_csr_create.
 *   MONOMIAL  theta = 0, sigma = max(|lo|, |hi|)          (the paper's choice, Sec. VI)
 *   SHIFTED   theta = (lo+hi)/2, sigma = (hi-lo)/2
 *   NEWTON    theta_i = newton_shifts[i] (host), sigma = (hi-lo)/2
 *   LEJA      Newton basis from Ritz values (the better-conditioned basis the paper names
 *             for larger s, Sec. IV and Sec. VI, after Bai, Hu and Reichel): cycles run
 *             with SHIFTED until one keeps >= s columns; at its end the device computes
 *             the eigenvalues of that cycle's Hessenberg matrix (Francis double-shift QR),
 *             Leja-orders them (conjugates adjacent) and takes the first s in real form
 *             (a pair a +- ib as theta = a, a and tau = b^2 / sigma on its second step),
 *             sigma = the capacity estimate of the ordered Ritz values; every later cycle
 *             uses them (tsg_solve_info.newton_from_cycle).  Not used by CGS2.          */
typedef enum {
  TSG_BASIS_MONOMIAL = 0,
  TSG_BASIS_SHIFTED = 1,
  TSG_BASIS_NEWTON = 2,
  TSG_BASIS_LEJA = 3
} tsg_basis;

/* FP64: every step in float64.
 * FP32_IR: basis, SpMV and tall-skinny products in float32 with float32
 * accumulation; Gram Cholesky, Hessenberg/Givens least squares, solution update
 * and the outer residual r = b - A x in float64.  Each restart cycle is one step of
 * iterative refinement (not in the paper). */
typedef enum { TSG_PREC_FP64 = 0, TSG_PREC_FP32_IR = 1 } tsg_prec;

typedef struct {
  int32_t m;            /* restart length (Krylov vectors per cycle), 1 <= m <= 63      */
  int32_t s;            /* step size; s divides m; 1 <= s <= 16 (CGS2 ignores s)        */
  int32_t s_hat;        /* two-stage big-panel size: 0 or m (one stage 2 per cycle), or
                           s | s_hat | m (stage 2 = BCGS-PIP of every completed big panel
                           against the final columns, explicit Q; the residual is checked
                           at every big-panel end)                                      */
  int32_t ortho;        /* tsg_ortho                                                    */
  int32_t basis;        /* tsg_basis                                                    */
  int32_t precision;    /* tsg_prec                                                     */
  double tol;           /* stop when ||b - A x||_2 <= tol ||b||_2 (explicit, FP64)      */
  int64_t max_iters;    /* stop (TSG_NOT_CONVERGED) once this many vectors were built   */
  const double* newton_shifts; /* host, length s, only for TSG_BASIS_NEWTON             */
  int32_t timing;       /* 0: off.  t >= 1: time each launch of every t-th restart cycle
                           (cycles 0, t, 2t, ...) with HIP events; timed cycles are
                           launched directly even in graph mode                         */
  int32_t flags;        /* TSG_FLAG_* bits, 0 by default                                */
  int32_t precond;      /* tsg_precond: right preconditioning (FP64 only)               */
} tsg_solve_params;

/* Right preconditioning (the paper's last experiment, Sec. VI, Fig. 13, runs s-step GMRES
 * with a local Gauss-Seidel preconditioner swept by colors on the GPU).  GMRES runs on
 * A M^{-1}: every matrix-powers step applies z = M^{-1} w then A z, the cycle update is
 * x += M^{-1} (Q y), and the residual stays the true one.
 *   NONE  no preconditioner
 *   MCGS  M = D + L_c, one forward multicolor Gauss-Seidel sweep from z = 0 (colors from
 *         tsg_csr_precond); the basis interval [lo, hi] becomes [0, 2] (the eigenvalues
 *         of A M^{-1} lie in |z - 1| < 1 for a convergent Gauss-Seidel splitting) */
typedef enum { TSG_PRECOND_NONE = 0, TSG_PRECOND_MCGS = 1 } tsg_precond;

/* tsg_solve_params.flags.  By default the launches of one restart cycle (they are the
 * same in every cycle) are captured once per solve into a HIP graph on a private
 * stream and the graph is replayed on `stream` once per cycle (HIP events cannot be
 * captured as timing nodes here, so cycles timed by params.timing are enqueued
 * directly).
 *   EAGER  launch every kernel of every cycle directly on `stream` instead (same
 *          kernels and arguments, bitwise-identical results).
 * Two-stage cycles run first without stage 1's fallback passes (the launches that only
 * check whether a panel needs them); a cycle whose PIP pivot test fails there ends at once,
 * before it has touched x or the counters, and is run again with the full sequence, which
 * runs from then on (tsg_solve_info.redone_cycles).  The results are the same bit for bit. */
enum { TSG_FLAG_EAGER = 1 };

/* Kernel classes reported by tsg_solve_info (timing mode).  Each class is one kernel
 * instantiation for a given precision and step size s. */
enum {
  TSG_KC_MPK = 0,        /* one step of the matrix-powers kernel (SpMV)                  */
  TSG_KC_GRAM = 1,       /* panel reduction (two-stage: with the previous panel's Gram)   */
  TSG_KC_GRAM_FIRST = 2, /* panel reduction of the first panel of a cycle                 */
  TSG_KC_UPDATE = 3,     /* panel update W <- (W - Q P) T                                 */
  TSG_KC_FUSED = 4,      /* panel update that also reduces the Gram of its output         */
  TSG_KC_TAIL = 5,       /* one-block FP64 tail of a reduction                            */
  TSG_KC_CYCLE_END = 6,  /* stage 2 / projected least squares                             */
  TSG_KC_XUPDATE = 7,    /* x += V coef                                                   */
  TSG_KC_RESIDUAL = 8,   /* r = b - A x and its tail                                      */
  TSG_KC_SCALE = 9,      /* first basis vector r / beta                                   */
  TSG_KC_FALLBACK = 10,  /* two-stage explicit second pass (its launches return at entry
                            unless a panel needs it; no bytes are attributed)            */
  TSG_KC_STAGE2 = 11,    /* two-stage with s_hat < m: big-panel stage 2 (tail, explicit Q) */
  TSG_KC_PRECOND = 12,   /* multicolor Gauss-Seidel sweeps of right preconditioning       */
  TSG_KC_COUNT = 13
};

typedef struct {
  int64_t iters;        /* Krylov vectors generated (the paper's iteration count)       */
  int64_t cycles;       /* restart cycles run                                           */
  double relres;        /* explicit ||b - A x|| / ||b|| of the returned x (FP64)         */
  double relres_est;    /* implicit estimate at the end of the last cycle               */
  int32_t status;       /* tsg_status of the solve                                      */
  int32_t truncated_cycles; /* cycles shortened by a Cholesky breakdown                 */
  /* filled only when params.timing != 0 (milliseconds of GPU time, HIP events); every
   * per-class figure is a total over the timed cycles only; ms_total spans the solve */
  double ms_total, ms_spmv, ms_ortho_reduce, ms_ortho_update, ms_small, ms_xupdate, ms_residual;
  int64_t n_ortho_reduce, n_ortho_update, n_spmv;  /* launches of each class           */
  double bytes_ortho_reduce, bytes_ortho_update, bytes_spmv; /* algorithmic bytes moved */
  double kc_ms[16];        /* per kernel class (TSG_KC_*): GPU milliseconds               */
  int64_t kc_launches[16]; /* launches that did work                                      */
  double kc_bytes[16];     /* algorithmic bytes (sum over launches)                       */
  int64_t timed_cycles;    /* restart cycles whose launches were timed                    */
  int64_t pip_fallbacks;   /* two-stage: stage-1 panels whose Pythagorean Gram failed the
                              pivot test and took the explicit second pass              */
  int64_t newton_from_cycle; /* LEJA: cycles completed when the Newton basis took over
                                (0: it never did)                                       */
  int64_t shifted_passes;  /* two-stage with s >= 8 or FP32_IR: stage-1 panels whose
                              explicit second pass failed too and took the shifted Cholesky
                              QR pass (Fukaya et al.; Sec. II names it as CholQR's remedy):
                              Rs = Chol(G + mu I), mu = 10 pivot_tol trace(G), then one
                              more BCGS-PIP pass; elsewhere such a panel ends the cycle */
  int64_t redone_cycles;   /* two-stage: restart cycles run first without stage 1's fallback
                              passes (the launches that check for them), met a panel that needs
                              them, and were run again in full; the full cycle runs from then on
                              (the results are the same bit for bit either way)             */
} tsg_solve_info;

typedef struct tsg_csr_s* tsg_csr;

/* Create a handle for the n x n CSR matrix (Sec. VII: the operator).  The handle
 * BORROWS row_ptr[n+1], col[nnz], val[nnz] (device): they must stay valid and
 * unchanged until tsg_csr_destroy.  Computes the Gershgorin interval and the plan of the
 * packed layout on the device (small kernels, synchronizes `stream`; their temporaries are
 * stream-ordered allocations freed before it returns).  The handle owns one 4 KiB device
 * block and about n/8 bytes of host memory.
 * Errors: INVALID_ARG for n < 1, nnz < 0, nnz >= 2^31, NULL pointers; HIP. */
tsg_status tsg_csr_create(int64_t n, int64_t nnz, const int32_t* row_ptr, const int32_t* col,
                          const double* val, void* stream, tsg_csr* out /* host */);
tsg_status tsg_csr_destroy(tsg_csr A);
/* Gershgorin interval [lo, hi] (host outputs). */
tsg_status tsg_csr_gershgorin(tsg_csr A, double* lo, double* hi);

/* Packed layout of the operator for the solver's SpMVs (optional, recommended): SELL-64 --
 * slices of 64 rows stored entry by entry, so one wave reads its slice's values and
 * columns as contiguous 64-entry runs and no row pointers; columns as int16 deltas
 * col - row when all fit, else int32; FP64 values and their FP32 copy (mixed form).
 * tsg_csr_pack_bytes: device bytes needed (the layout plan is computed at create).
 * tsg_csr_pack: fill buf (device, 256-byte aligned, caller-owned, must stay valid while
 * the handle uses it) from the CSR arrays, asynchronously on `stream`; from then on every
 * solve with A uses the packed copy (the CSR arrays must still stay valid).  buf = NULL
 * returns to the CSR arrays (synchronizes `stream`).  The packed SpMV sums each row's
 * products in CSR order, rounded as the CSR kernel rounds them: results are identical. */
size_t tsg_csr_pack_bytes(tsg_csr A);
tsg_status tsg_csr_pack(tsg_csr A, void* buf, size_t bytes, void* stream);

/* Multicolor Gauss-Seidel set-up for TSG_PRECOND_MCGS: a distance-1 coloring of the
 * pattern by Jones and Plassmann's parallel rounds (priority of row i = output i of the
 * SplitMix64 generator seeded with 0, ties to the higher index; equal to the greedy
 * coloring in decreasing priority), the order P (blocks of 8192 consecutive rows; within
 * a block the rows grouped by color, index order within a color: counting sort of the
 * device-computed colors on the host), the reordered system P A P^T (CSR with columns
 * renamed and sorted, its own Gershgorin interval and packed copy) on which
 * preconditioned solves run, and its sweep layout: the rows of one color within one block
 * cut into slices of 64 with their lower-color entries stored entry by entry.
 * tsg_csr_precond_bytes: device bytes of the buffer, an upper bound from n, nnz and the
 * longest row of every block of 8192 rows (known since tsg_csr_create): about
 * 12 nnz + (60 + 28 W) n bytes for rows of at most W entries; 0 for a NULL handle.
 * tsg_csr_precond: everything the set-up builds or uses lives in buf (device, 256-byte
 * aligned, caller-owned, at least tsg_csr_precond_bytes(A) bytes; it must stay valid and
 * untouched until tsg_csr_destroy): the library allocates no device memory (the internal
 * handle of P A P^T takes its 4 KiB block from buf too).  Synchronizes `stream`; a second
 * call does nothing.  The pattern must be structurally symmetric (a_ij stored iff a_ji
 * stored) and every row must store a nonzero diagonal.  From then on solves with
 * precond = MCGS may use A.  Errors: INVALID_ARG (NULL handle or buffer); WORKSPACE
 * (misaligned or too small); UNSUPPORTED when the rounds do not finish within n rounds;
 * HIP (launches, copies). */
size_t tsg_csr_precond_bytes(tsg_csr A);
tsg_status tsg_csr_precond(tsg_csr A, void* buf, size_t bytes, void* stream);
/* Number of colors of the preconditioner set-up (0 before tsg_csr_precond). */
int32_t tsg_csr_ncolors(tsg_csr A);
/* Copy the n row colors (int32) to colors (device, caller-owned); INVALID_ARG before
 * tsg_csr_precond. */
tsg_status tsg_csr_colors(tsg_csr A, int32_t* colors, void* stream);

/* z = M^{-1} w for the handle's multicolor Gauss-Seidel preconditioner (device vectors of
 * n doubles; z must not alias w): w is put in the order of P A P^T, swept as in the solver's
 * matrix-powers steps, and z put back.  Uses two scratch vectors of the handle: calls on
 * one handle must not overlap. */
tsg_status tsg_precond_apply(tsg_csr A, const double* w, double* z, void* stream);

/* Newton-basis parameters of TSG_BASIS_LEJA for a given k x k upper Hessenberg matrix
 * H (device, column-major, leading dimension ldh >= k; entries below the subdiagonal are
 * ignored), 1 <= s <= k <= 63: the same device routine the solver runs at a cycle end.
 * out (device, 2k + 3s + 1 doubles, caller-owned): the Ritz values in Leja order (k real
 * parts, then k imaginary parts), theta (s), tau (s), sigma (s), then a status word.
 * [lo, hi] supplies the fallback scaling (hi - lo) / 2.  Synchronizes `stream`.
 * Returns TSG_BREAKDOWN (status word 1) when the QR iteration did not converge within
 * 30 k double-shift steps; INVALID_ARG for bad sizes or NULL pointers; HIP. */
tsg_status tsg_ritz_newton(const double* H, int64_t ldh, int32_t k, int32_t s, double lo, double hi, double* out,
                           void* stream);

/* y = A x in float64 (the SpMV of the matrix-powers kernel with theta = 0, sigma = 1).
 * x and y must not overlap.  Asynchronous on `stream`. */
tsg_status tsg_spmv(tsg_csr A, const double* x, double* y, void* stream);

/* Workspace (device, 256-byte aligned) needed by tsg_solve for this matrix and params. */
size_t tsg_solve_workspace_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p);

/* Solve A x = b by restarted s-step GMRES(m) (Sec. III, Fig. 1) with the block
 * orthogonalization p->ortho.  b[n] (device, float64) is read; x[n] (device, float64)
 * holds x0 on entry and the result on exit.  Every step of a restart cycle runs in
 * the library's HIP kernels on `stream`; the host only reads back an 80-byte status
 * block once per cycle (the host synchronizes `stream` once per cycle).  Returns after
 * the solve has finished on the device.  precond = MCGS: the solve runs on the operator's
 * reordered system P A P^T (b and x permuted in and out on `stream`).
 * Status: OK (converged), NOT_CONVERGED, BREAKDOWN, or a negative error (then x is
 * untouched).  `info` (host) is filled for every non-negative status. */
tsg_status tsg_solve(tsg_csr A, const double* b, double* x, const tsg_solve_params* p,
                     void* workspace, size_t ws_bytes, void* stream,
                     tsg_solve_info* info /* host, may be NULL */);

/* Workspace (device) needed by tsg_orthogonalize for an n x k block with step s. */
size_t tsg_orthogonalize_workspace_bytes(int64_t n, int32_t k, int32_t s);

/* Orthonormalize the tall-skinny block X (n x k, column-major, leading dimension
 * ldx >= n, device float64) in place:  on exit X holds Q with X_in = Q R, Q^T Q = I,
 * R upper triangular with positive diagonal (the contract of Fig. 1's caption).
 * Column 1 is normalized alone; then panels of s columns (the last may be short).
 * algo: TWO_STAGE (stage 1 = BCGS-PIP per panel, stage 2 = one CholQR over all k
 * columns, then Q = Qhat R2^{-1}), BCGS_PIP2 or BCGS2_CHOLQR2.  s_hat (TWO_STAGE): 0 or
 * >= k-1 for one big panel; else a multiple of s: big panels of s_hat columns (the first
 * also holds column 1, the last may be short), each orthogonalized by stage 2 = BCGS-PIP
 * against the final columns before it, its Q made explicit before the next big panel's
 * stage 1 (Sec. V, Fig. 5; stage 1 projects every panel against all earlier columns).  R (device, k x k, column-major, leading dimension ldr >= k) receives R; its
 * strictly lower part is set to 0.  Requires 1 <= k <= 64, 1 <= s <= 16, k <= n.
 * Synchronizes `stream` before returning (the breakdown status is read back).  If
 * orth_err (host) is non-NULL, ||I - Q^T Q||_F is also computed on the device (one
 * extra pass) and returned.
 * Status BREAKDOWN: a Gram matrix was not numerically positive definite (X is then
 * partially overwritten). */
tsg_status tsg_orthogonalize(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr,
                             int32_t s, int32_t s_hat, int32_t algo, void* workspace,
                             size_t ws_bytes, void* stream, double* orth_err /* host, opt */);

/* One stage-1 panel of the two-stage scheme through the solver's fallback chain
 * (Sec. V, Fig. 5 stage 1; Sec. IV-C, Fig. 4a for BCGS-PIP and its stability limit; Sec. II
 * names shifted Cholesky QR as the remedy for CholQR's breakdown): W = V(:, k:k+s) is
 * orthogonalized against Q = V(:, 0:k) (device float64, column-major, ldv >= n; Q is taken
 * as given, normally orthonormal) and overwritten by Qnew with W = Q P + Qnew R.
 *   pass 0  BCGS-PIP: one reduction [Q, W]^T W, R = Chol(W^T W - P^T P); a relative pivot
 *           R_jj^2 <= pip_tol (W^T W)_jj fails the pass (the solver uses 1e-8 in FP64);
 *   pass 1  (chain >= 1, only if pass 0 failed) the explicit second pass: Y = W - Q P1,
 *           then BCGS-PIP of Y; a pivot fails at <= max(pivot_tol (Y^T Y)_jj,
 *           pivot_tol^2 (W^T W)_jj) (the solver uses pivot_tol = 1e-12);
 *   pass 2  (chain = 2, only if pass 1 failed) shifted Cholesky QR of pass 1's Gram G,
 *           Rs = Chol(G + mu I), mu = 10 pivot_tol trace(G), Z = (Y - Q P2) Rs^{-1}, then
 *           BCGS-PIP of Z; a final (R3 Rs)_jj^2 <= pivot_tol^2 (W^T W)_jj still fails.
 * The kernels and tails are the solver's own (the same reductions, updates and gates).
 * P (device, k x s, ldp >= k; unused when k = 0) and R (device, s x s upper triangular,
 * ldr >= s, strictly lower part set to 0) receive the factors.  out (host, 2 ints,
 * optional): out[0] = the last pass taken (0, 1 or 2), out[1] = the failing column of the
 * panel on BREAKDOWN, else -1.  Requires 0 <= k, 1 <= s <= 16, k + s <= min(n, 64),
 * 0 <= pip_tol, pivot_tol < 1, pivot_tol > 0 when chain >= 1.  Workspace (device, 256-byte
 * aligned): tsg_block_pip_workspace_bytes.  Synchronizes `stream`.  BREAKDOWN: the last
 * pass of the chain failed (W is then partially overwritten and P, R are not written);
 * INVALID_ARG, WORKSPACE, HIP as elsewhere. */
size_t tsg_block_pip_workspace_bytes(int64_t n, int32_t k, int32_t s);
tsg_status tsg_block_pip(int64_t n, int32_t k, int32_t s, double* V, int64_t ldv, double pip_tol,
                         double pivot_tol, int32_t chain, double* P, int32_t ldp, double* R, int32_t ldr,
                         int32_t* out /* host, 2, opt */, void* workspace, size_t ws_bytes, void* stream);

/* For callers that cannot allocate device memory (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): tsg_orthogonalize without a workspace
 * argument.  Same arguments, layout, results (bit for bit) and status codes as
 * tsg_orthogonalize; the workspace is instead a file-scope device array of
 * tsg_orthogonalize_noalloc_max_bytes() = 12 MiB that every GPU the library runs on holds
 * until the process ends (its address on the current device is looked up once, on the first
 * call there).  The call makes no device allocation.  Limits: n <= 268,435,456 rows (and the
 * limits of tsg_orthogonalize); larger n returns INVALID_ARG with a message, before any device
 * work.  Every call on one GPU shares that GPU's array: calls that overlap on one GPU (other
 * host threads, or other streams before this call has returned) race and give wrong results;
 * the call synchronizes `stream` before returning, so calls made one after another from one
 * thread are safe.  X, R and `stream` must belong to the current device. */
size_t tsg_orthogonalize_noalloc_max_bytes(void);
tsg_status tsg_orthogonalize_noalloc(int64_t n, int32_t k, double* X, int64_t ldx, double* R, int32_t ldr,
                                     int32_t s, int32_t s_hat, int32_t algo, void* stream,
                                     double* orth_err /* host, opt */);

/* ---------------------------------------------------------------- solve server
 * Continuous batching of many solves (different operators and sizes) that share one
 * tsg_solve_params (m, s, ortho, basis monomial or shifted, precision, tol, max_iters;
 * timing must be 0).  Requests wait in a FIFO queue; at every restart-cycle boundary
 * tsg_server_step admits queued requests in arrival order while their buffers fit the
 * arena and a slot is free (a request that does not fit blocks the ones behind it), runs
 * ONE restart cycle of every active request -- each kernel of the cycle is one launch over
 * all of them -- and retires the finished ones, whose memory serves the queue next.  A
 * request computes bit for bit what tsg_solve computes for it (its launches use its own
 * buffers and block decomposition whatever else is batched).  Not thread-safe: one host
 * thread drives a server. */
typedef struct tsg_server_s* tsg_server;

/* Arena bytes one request occupies while active (its admission footprint): reduction
 * buffers and state, the (m+1)-column basis, and the FP32 copy of the values in the mixed
 * form.  0 for invalid arguments. */
size_t tsg_server_request_bytes(int64_t n, int64_t nnz, const tsg_solve_params* p);

/* Create a server.  arena (device, 256-byte aligned, arena_bytes) is caller-owned and must
 * outlive the server: it holds the launch image of up to max_active requests (512 KiB
 * each), their status heads, and every admitted request's buffers (the HBM budget).  The
 * server makes no device allocation; it owns one pinned host buffer of max_active x 72
 * bytes.  All device work goes to `stream`.  Errors: INVALID_ARG (bad params, max_active
 * outside [1, 4096]), UNSUPPORTED (timing, a Newton basis, or a preconditioner), WORKSPACE (arena misaligned
 * or smaller than the launch images plus 1 MiB). */
tsg_status tsg_server_create(const tsg_solve_params* p, void* arena, size_t arena_bytes, int32_t max_active,
                             void* stream, tsg_server* out /* host */);
tsg_status tsg_server_destroy(tsg_server S);

/* Queue the solve of A x = b.  b[n] and x[n] are device float64 (x holds x0); they and the
 * CSR handle must stay valid until the request is returned by tsg_server_poll.  tag is the
 * caller's identifier.  INVALID_ARG if the request could never fit the arena. */
tsg_status tsg_server_submit(tsg_server S, tsg_csr A, const double* b, double* x, int64_t tag);

/* One restart-cycle boundary: admission, one cycle of every active request, retirement.
 * Synchronizes the stream (one read-back of all status heads).  n_active / n_queued
 * (host, optional) receive the counts afterwards. */
tsg_status tsg_server_step(tsg_server S, int32_t* n_active, int32_t* n_queued);

/* Remove up to max finished requests: tags[i] (host) and infos[i] (host, may be NULL;
 * iteration counts, residuals and status as from tsg_solve).  Returns how many. */
int32_t tsg_server_poll(tsg_server S, int64_t* tags, tsg_solve_info* infos, int32_t max);

const char* tsg_status_string(tsg_status st);
const char* tsg_last_error(void);

#ifdef __cplusplus
}
#endif
#endif /* TSGMRES_H */
