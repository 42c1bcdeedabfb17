/*
 * rorbk.h -- C ABI of the MI355X ROR-BK library.
 *
 * ROR-BK (Regularized Orthogonality and Residual based Block-Kaczmarz;
 * Kar & Venkatapathi, arXiv 2510.02156, Algorithm 1) solves a consistent
 * system A x = b, A in R^{m x n} of any shape (Section 1, the linear system;
 * Section 2), dense row-major or CSR.  Setup cuts A into k contiguous row
 * blocks, scores each block by its centroid's cosine with every other centroid
 * and stores the inverse of every regularised block Gram.  Each outer iteration
 * makes three sampled block updates x += A_t^T (A_t A_t^T + lambda I)^{-1}
 * (b_t - A_t x), a full residual pass with the stop test, and one greedy update
 * on the rows of largest |r_i|.
 *
 * Conventions for every entry point:
 *  - Matrix, right-hand side, iterate and gradient buffers are DEVICE memory
 *    owned by the caller.  The handle keeps non-owning pointers to the matrix
 *    arrays, which must stay valid and unchanged until ror_bk_destroy.
 *  - Arrays named "_host" are host memory owned by the caller.
 *  - All device work is enqueued on the stream given to ror_bk_setup (NULL =
 *    the default stream).  Calls that return values to the host synchronise
 *    that stream before they return.
 *  - Functions return 0 (RORBK_OK) or one of the RORBK_ERR_* codes; no
 *    exception crosses the ABI and nothing exits the process.
 *    ror_bk_last_error_message() describes the last failure of the calling
 *    thread.  Non-convergence is not an error (rorbk_info.converged == 0).
 *  - A handle is not thread safe; distinct handles are independent.
 *
 * Vector types: in FP64 solves (matrix dtype F64, or any dtype with
 * RORBK_REFINE) b, x and the gradients are double.  A solve on an F32 or BF16
 * matrix without RORBK_REFINE uses float vectors (FP32 passes with FP32
 * accumulation; block Gram, Cholesky and solves stay FP64).
 */
#ifndef RORBK_H
#define RORBK_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

/* ------------------------------------------------------------ status codes */
#define RORBK_OK 0
#define RORBK_ERR_INVALID_ARG 1  /* bad shape, pointer, size or flag          */
#define RORBK_ERR_OOM 2          /* device or host allocation failed         */
#define RORBK_ERR_HIP 3          /* a HIP runtime call failed                 */
#define RORBK_ERR_NOT_SPD 4      /* a block Gram A_t A_t^T + lambda I was not
                                    positive definite (lambda = 0 with a
                                    rank-deficient block)                     */
#define RORBK_ERR_NONFINITE 5    /* NaN or Inf in the residual               */
#define RORBK_ERR_NOT_RECORDED 6 /* backward without a recorded forward      */
#define RORBK_ERR_UNSUPPORTED 7  /* valid but not implemented (a block larger
                                    than the limits below)                    */

/* Largest rows per block (blocks may carry one extra row): CSR storage takes
 * blocks of up to RORBK_MAX_BLOCK_ROWS + 1 rows; dense storage also takes
 * larger blocks, of up to RORBK_MAX_BIG_BLOCK_ROWS rows, through a path built
 * for them (blocked factorisations and multi-workgroup block steps). */
#define RORBK_MAX_BLOCK_ROWS 160
#define RORBK_MAX_BIG_BLOCK_ROWS 2048

/* ------------------------------------------------------------------ matrix */
#define RORBK_DENSE 0
#define RORBK_CSR 1
#define RORBK_F64 0
#define RORBK_F32 1
#define RORBK_BF16 2 /* 16-bit storage: the upper half of an IEEE float */

typedef struct rorbk_matrix {
    int32_t format;            /* RORBK_DENSE or RORBK_CSR                     */
    int32_t dtype;             /* RORBK_F64, RORBK_F32 or RORBK_BF16 (dense)  */
    int64_t m, n;              /* rows, columns (m >= 1, n >= 1)               */
    int64_t ld;                /* dense: row stride in elements (ld >= n)      */
    const void *values;        /* dense: m*ld entries; CSR: nnz entries        */
    const int64_t *rowptr;     /* CSR: m+1 offsets, rowptr[0] = 0              */
    const int32_t *colidx;     /* CSR: nnz column indices, ascending per row   */
    int64_t nnz;               /* CSR: number of stored entries                */
    const double *values_f64;  /* optional FP64 master copy with the same
                                  layout; required by RORBK_REFINE when dtype
                                  is not F64 (ignored otherwise)               */
} rorbk_matrix;

/* --------------------------------------------------------------- solve info */
typedef struct rorbk_info {
    int64_t iters;       /* outer iterations run (inner ones under REFINE)   */
    double rrn;          /* last measured ||b - A x|| / ||b||                 */
    int32_t converged;   /* 1 if rrn < tol was reached                         */
    int32_t n_refine;    /* REFINE: outer FP64 correction steps               */
    double t_solve_s;    /* device time of the solve (HIP events)             */
} rorbk_info;

typedef struct rorbk_handle_s *rorbk_handle;

/* Solve flags */
#define RORBK_REFINE 1u      /* FP32/BF16 inner passes + FP64 refinement      */
#define RORBK_RECORD 2u      /* keep tau and the greedy sets for backward     */
#define RORBK_REPLAY 4u      /* take tau and the greedy sets from set_replay  */
#define RORBK_CHECKPOINT 8u  /* keep x every checkpoint_every iterations and
                                recompute the greedy sets during backward     */
#define RORBK_PROFILE 16u    /* time the residual-pass kernel with HIP events
                                (one launch in every 16 iterations, plus every
                                FP64 outer pass); read with ror_bk_get_profile */

/* Setup (Algorithm 1, first four steps; Section 3.1 for the stored block
 * inverses).  Partitions A into k = floor(m / block_rows) contiguous blocks of
 * floor(m/k) or floor(m/k)+1 rows (the first m mod k blocks take the extra
 * row), forms the block centroids (sums of rows), the cosine row sums
 * S_t = sum_j |<c_t,c_j>| / (|c_t| |c_j|), the proposal Pbar_t = exp(-2 S_t / n)
 * with its running sums W, and the inverse (A_t A_t^T + lambda I)^{-1} of every
 * block.  lambda >= 0 (the paper uses 1e-6 * rows per block; lambda = 0 needs
 * every block to have full row rank, else RORBK_ERR_NOT_SPD).
 * stream: a hipStream_t or NULL.  On success *out owns all device workspaces. */
int ror_bk_setup(const rorbk_matrix *A, int64_t block_rows, double lambda,
                 void *stream, rorbk_handle *out);

/* Run ROR-BK (Algorithm 1) from the iterate in x (device, length n; updated in
 * place) against b (device, length m).  Outer iteration j (j = start_iter ..
 * start_iter + max_iters - 1) draws its three blocks from word 3j + l - 1 of a
 * counter-based SplitMix64 stream keyed by seed, by inverse CDF over W; then
 * computes r = b - A x and stops when ||r|| < tol * ||b|| (before the greedy
 * step); otherwise it updates on the floor(m/k) rows of largest |r_i| (ties to
 * the lower index).  tol = 0 runs exactly max_iters iterations.
 * flags: RORBK_REFINE (needs the FP64 master copy for non-F64 storage; not
 * combinable with RECORD, REPLAY or CHECKPOINT), RORBK_RECORD, RORBK_REPLAY,
 * RORBK_CHECKPOINT (checkpoint_every >= 1).  info may be NULL. */
int ror_bk_solve(rorbk_handle h, const void *b, void *x, uint64_t seed,
                 double tol, int64_t max_iters, int64_t start_iter,
                 uint32_t flags, int64_t checkpoint_every, rorbk_info *info);

/* Reverse-mode derivative of the last RECORD or CHECKPOINT solve.  With the
 * sampled and greedy selections held fixed, each block step x' = x +
 * A_S^T H_S (b_S - A_S x), H_S = (A_S A_S^T + lambda I)^{-1}, is linear in
 * (x, b) (the update rule of Lemma 2), so its adjoint is y = H_S A_S g',
 * gb[S] += y, g = g' - A_S^T y, taken newest step first.  grad_x (device, n)
 * holds dL/dx_final; grad_b (device, m) and grad_x0 (device, n) receive dL/db
 * and dL/dx0.  The b used by the forward must still be valid for CHECKPOINT
 * (it is read again to recompute the greedy sets).  RORBK_ERR_NOT_RECORDED if
 * no recorded solve precedes. */
int ror_bk_backward(rorbk_handle h, const void *grad_x, void *grad_b,
                    void *grad_x0);

/* Release every device buffer of the handle (h may be NULL). */
int ror_bk_destroy(rorbk_handle h);

/* ------------------------------------------------- inspection and replay -- */

/* Sizes chosen by setup: k blocks, K greedy rows, largest block rows. */
int ror_bk_get_sizes(rorbk_handle h, int64_t *k, int64_t *K, int64_t *bmax);

/* Copies of the setup results: offsets (k+1 int64), S, Pbar, W (k doubles
 * each).  Any pointer may be NULL. */
int ror_bk_get_setup(rorbk_handle h, int64_t *offsets_host, double *S_host,
                     double *pbar_host, double *W_host);

/* Replace the sampler's running sums W (k doubles, host), e.g. with another
 * implementation's table so that sampled indices can be compared bit for bit. */
int ror_bk_set_proposal(rorbk_handle h, const double *W_host);

/* Which form of the regularised block solve setup chose (Sec. 3.1): 0 for the
 * row form, A_t^T (A_t A_t^T + lambda I)^{-1}, with b_t x b_t stored inverses;
 * 1 for the column form, (A_t^T A_t + lambda I)^{-1} A_t^T, taken for dense
 * blocks of more than RORBK_MAX_BLOCK_ROWS + 1 rows that have at least as many
 * rows as columns, with n x n stored inverses.  Both compute the same update
 * (Lemma 1), and ror_bk_backward differentiates either. */
int ror_bk_get_form(rorbk_handle h, int32_t *column_form);

/* The stored inverse of block t into host memory, row-major doubles: row
 * form (A_t A_t^T + lambda I)^{-1}, b_t x b_t; column form
 * (A_t^T A_t + lambda I)^{-1}, n x n. */
int ror_bk_get_block_inverse(rorbk_handle h, int64_t t, double *Hinv_host);

/* The block indices the sampler draws for iterations j0 .. j0+count-1
 * (3 per iteration, draw l of iteration j at [3(j-j0) + l - 1]), computed on
 * the device, copied to tau_host (3*count int32). */
int ror_bk_sample(rorbk_handle h, uint64_t seed, int64_t j0, int64_t count,
                  int32_t *tau_host);

/* The greedy selection on a given residual: the K indices of largest |r_i|
 * (ties to the lower index), ascending.  r: device, m entries of the solve's
 * vector type (vec_f32 = 0: double, 1: float).  idx: device, K int32. */
int ror_bk_topk(rorbk_handle h, const void *r, int32_t vec_f32, int32_t *idx);

/* One residual pass r = b - A x with the per-block squared norms
 * ||r_t||^2 (block_norm2, device, k doubles) and ||r|| / ||b|| in *rrn_host.
 * b, x, r: device, of the vector type given by vec_f32 (0: double; 1: float,
 * only for F32/BF16 storage).  use_f64_master = 1 reads the FP64 master copy. */
int ror_bk_residual(rorbk_handle h, const void *b, const void *x, void *r,
                    double *block_norm2, int32_t vec_f32,
                    int32_t use_f64_master, double *rrn_host);

/* Selections of the last RECORD (or CHECKPOINT-recomputed) solve: tau
 * (3*iters int32), greedy sets (iters*K int32), RRN history (iters doubles),
 * each pointer may be NULL; *iters_host receives the iterations recorded. */
int ror_bk_get_record(rorbk_handle h, int32_t *tau_host, int32_t *I_host,
                      double *rrn_host, int64_t *iters_host);

/* Selections for a RORBK_REPLAY solve of up to `iters` iterations: tau
 * (3*iters int32, block indices in [0,k)), greedy sets (iters*K int32, row
 * indices in [0,m), ascending within a set), host memory, copied. */
int ror_bk_set_replay(rorbk_handle h, const int32_t *tau_host,
                      const int32_t *I_host, int64_t iters);

/* Flexible AB-GMRES with ROR-BK as the right preconditioner (appendix,
 * Algorithm 3, and the remark on it in Section 2).  FP64 storage; b (device,
 * m doubles), x (device, n doubles: x0 in, result out).  From r0 = b - A x0:
 * outer step k runs ROR-BK (Algorithm 1, this handle's setup) on A z = v_k
 * from z = 0 for at most inner_iters iterations, stopping once
 * ||v_k - A z|| < eta ||v_k|| (draws from words of the seed's stream starting
 * at iteration k * inner_iters), orthogonalises w = A z_k against v_1..v_k by
 * modified Gram-Schmidt, and reduces the Hessenberg least-squares problem with
 * Givens rotations; it stops when that problem's residual is below
 * tol * ||b||, on breakdown, or after max_outer steps; then x = x0 + Z y.
 * info (may be NULL): iters = inner iterations in total, n_refine = outer
 * steps, converged, rrn = ||b - A x|| / ||b|| of the result.  Workspaces of
 * (m + n) * (max_outer + 1) doubles are allocated for the call. */
int ror_bk_fabgmres(rorbk_handle h, const double *b, double *x, uint64_t seed, double tol,
                    int64_t max_outer, int64_t inner_iters, double eta, rorbk_info *info);

/* Initial solution (appendix, Algorithm 2, and the remark after it):
 * x0 = (<b, A y> / ||A y||^2) y with y the sum of all rows of A (kept from the
 * setup: the block row-sums added in block order), so that x0 lies in the row
 * space of A and ||b - A x0|| <= ||b||; x0 = 0 if A y = 0.  b (device, m) and
 * x0 (device, n, written) have the vector type given by vec_f32 (0: double,
 * with the FP64 master copy for F32/BF16 storage; 1: float, F32/BF16 storage
 * only).  coef_host (may be NULL) receives the coefficient; the stream is
 * synchronised only then.  Pass x0 as the starting iterate of ror_bk_solve. */
int ror_bk_initial_solution(rorbk_handle h, const void *b, void *x0, int32_t vec_f32,
                            double *coef_host);

/* Refinement controls for RORBK_REFINE: inner iterations per FP64 correction
 * (default 50) and the inner relative stop eta (default 1e-4; the inner solve
 * also stops once its residual is below tol * ||b||). */
int ror_bk_set_refine(rorbk_handle h, int64_t inner_iters, double eta);

/* Residual-pass timings of the last RORBK_PROFILE solve: out[0] = mean
 * duration (ms) of the sampled inner (working-precision) residual launches,
 * out[1] = their count, out[2] = mean duration (ms) of the FP64 outer residual
 * launches of a REFINE solve, out[3] = their count. */
int ror_bk_get_profile(rorbk_handle h, double *out4_host);

/* Static description of a status code. */
const char *ror_bk_error_string(int code);

/* Details of the calling thread's last failure ("" if none). */
const char *ror_bk_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* RORBK_H */
