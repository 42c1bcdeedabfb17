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
/* rrn is ||b - A x|| / ||b|| of the x the call returns, on every path: a
 * converged plain solve returns the iterate whose residual passed the stop
 * test (Algorithm 1 tests before the greedy step); a plain solve that ends at
 * max_iters made one greedy update after its last test, so one more residual
 * pass measures the returned x (in the solve's vector precision); REFINE
 * measures it in FP64 with the master copy.  rrn_test is the last stop test
 * of Algorithm 1 itself (the RRN history of ror_bk_get_record ends with it). */
typedef struct rorbk_info {
    int64_t iters;       /* outer iterations run (inner ones under REFINE)   */
    double rrn;          /* ||b - A x|| / ||b|| of the returned x             */
    int32_t converged;   /* 1 if the stop test ||r|| < tol ||b|| passed      */
    int32_t n_refine;    /* REFINE: outer FP64 correction steps               */
    double t_solve_s;    /* device time of the solve (HIP events)             */
    double t_setup_s;    /* wall time of the handle's ror_bk_setup call (s)   */
    double rrn_test;     /* RRN of the last stop test taken                   */
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

/* Block partition (Algorithm 1, first step; Section 2: k blocks of at least
 * floor(m/k) rows each), on the host, without a handle or any device work:
 * k = floor(m / block_rows) contiguous blocks; the first m mod k of them take
 * floor(m/k) + 1 rows, the others floor(m/k).  *k receives the block count;
 * offsets_host (host, caller-owned, may be NULL to query k) receives the k+1
 * row offsets, offsets_host[0] = 0 and offsets_host[k] = m, identical to the
 * partition ror_bk_setup builds on the device.  RORBK_ERR_INVALID_ARG unless
 * m >= 1 and 1 <= block_rows <= m (and k != NULL). */
int ror_bk_partition(int64_t m, int64_t block_rows, int64_t *offsets_host, int64_t *k);

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

/* Release every device buffer the handle owns (the stored block inverses of
 * Section 3.1, the proposal, workspaces and records); h may be NULL.  The
 * caller's matrix and vectors are not touched. */
int ror_bk_destroy(rorbk_handle h);

/* ------------------------------------------------- inspection and replay -- */

/* Sizes chosen by setup (Algorithm 1: k blocks from the first step; the
 * greedy step's floor(m/k) rows): k, K = floor(m/k), and the largest block's
 * rows.  Any pointer may be NULL (host, caller-owned). */
int ror_bk_get_sizes(rorbk_handle h, int64_t *k, int64_t *K, int64_t *bmax);

/* Copies of the setup results of Algorithm 1's first four steps into host
 * memory (caller-owned): the block offsets (k+1 int64, the partition), the
 * cosine row sums S_t = sum_j |<c_t,c_j>| / (|c_t| |c_j|) over the centroids
 * c_t (sums of the block's rows), Pbar_t = exp(-2 S_t / n) and the running
 * sums W_t = Pbar_0 + ... + Pbar_t the sampler inverts (k doubles each).  Any
 * pointer may be NULL.  Synchronises the stream. */
int ror_bk_get_setup(rorbk_handle h, int64_t *offsets_host, double *S_host,
                     double *pbar_host, double *W_host);

/* Replace the sampler's running sums W of the proposal (Algorithm 1, steps
 * 3-4: W_t = Pbar_0 + ... + Pbar_t; Section 2, sampling by the proposal):
 * W_host holds k doubles (host, copied), finite, non-negative and
 * non-decreasing, else RORBK_ERR_INVALID_ARG.  Lets another implementation's
 * table drive the draws, so that sampled indices can be compared bit for bit. */
int ror_bk_set_proposal(rorbk_handle h, const double *W_host);

/* Which form of the regularised block solve setup chose (Sec. 3.1): 0 for the
 * row form, A_t^T (A_t A_t^T + lambda I)^{-1}, with b_t x b_t stored inverses;
 * 1 for the column form, (A_t^T A_t + lambda I)^{-1} A_t^T, taken for dense
 * blocks of more than RORBK_MAX_BLOCK_ROWS + 1 rows that have at least as many
 * rows as columns, with n x n stored inverses.  Both compute the same update
 * (Lemma 1), and ror_bk_backward differentiates either. */
int ror_bk_get_form(rorbk_handle h, int32_t *column_form);

/* The stored inverse of block t (Section 3.1 keeps the inverse of every
 * fixed block's regularised Gram, so a sampled step costs O(nb)) into
 * Hinv_host (host, caller-owned), row-major doubles: row form
 * (A_t A_t^T + lambda I)^{-1}, b_t x b_t; column form
 * (A_t^T A_t + lambda I)^{-1}, n x n.  RORBK_ERR_INVALID_ARG if t is outside
 * [0, k).  Synchronises the stream. */
int ror_bk_get_block_inverse(rorbk_handle h, int64_t t, double *Hinv_host);

/* The sampled blocks of Algorithm 1's inner loop (three draws with
 * replacement per outer iteration, from the proposal P = Pbar / sum Pbar of
 * Section 2) for iterations j0 .. j0+count-1: draw l of iteration j uses word
 * 3j + l - 1 of the counter-based SplitMix64 stream keyed by seed and inverts
 * the running sums W (tau = number of W_t <= u W_{k-1}, at most k-1), at
 * [3(j-j0) + l - 1] of tau_host (host, caller-owned, 3*count int32).  Computed
 * on the device (a temporary buffer is allocated) and synchronised.
 * RORBK_ERR_INVALID_ARG if count < 0 or j0 < 0. */
int ror_bk_sample(rorbk_handle h, uint64_t seed, int64_t j0, int64_t count,
                  int32_t *tau_host);

/* The greedy step's selection of Algorithm 1 (the floor(m/k) rows of largest
 * r_i^2, the paragraph after the listing) on a given vector: the K indices of
 * largest |r_i| (ties to the lower index), ascending.  r: device, m entries
 * of the solve's vector type (vec_f32 = 0: double, 1: float), caller-owned,
 * read only.  idx: device, K int32, written.  Synchronises the stream;
 * RORBK_ERR_NONFINITE if r holds a NaN or Inf. */
int ror_bk_topk(rorbk_handle h, const void *r, int32_t vec_f32, int32_t *idx);

/* One full residual pass of Algorithm 1 (r = b - A x, the step before the
 * stop test; its O(mn) cost per iteration is the one Section 3.1 names) with
 * the per-block squared norms ||r_t||^2 (block_norm2, device, k doubles, may
 * be NULL) and ||r|| / ||b|| in *rrn_host (host, may be NULL).  b, x: device,
 * read; r: device, written; all of the vector type given by vec_f32 (0:
 * double; 1: float, only for F32/BF16 storage).  use_f64_master = 1 reads the
 * FP64 master copy (double vectors).  Synchronises the stream;
 * RORBK_ERR_NONFINITE if the residual holds a NaN or Inf. */
int ror_bk_residual(rorbk_handle h, const void *b, const void *x, void *r,
                    double *block_norm2, int32_t vec_f32,
                    int32_t use_f64_master, double *rrn_host);

/* Size of the static scratch array behind ror_bk_residual_noalloc (16 MiB,
 * one copy on each GPU the library runs on, held until the process ends). */
#define RORBK_NOALLOC_SCRATCH_BYTES 16777216

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): the
 * residual pass of ror_bk_residual without a handle and without any
 * allocation.  It runs the same kernels on the matrix described by A
 * (dense or CSR, not validated on the device: CSR arrays must be well formed)
 * partitioned as ror_bk_partition(A->m, block_rows) does, and enqueues on
 * `stream` (a hipStream_t or NULL) without synchronising:
 *   r = b - A x (device, written), block_norm2 (device, k doubles, may be
 *   NULL), *rrn = ||r|| / ||b|| (device, one double, may be NULL; NaN or Inf
 *   when the residual is not finite, as no status can be returned without a
 *   synchronisation).
 * b, x, r are of the vector type vec_f32 selects (0: double, reading A->values
 * for F64 storage, else A->values_f64; 1: float, F32 or BF16 storage).
 * Workspace: the static array (RORBK_NOALLOC_SCRATCH_BYTES) holds 1024 bytes
 * of control data, then 8 bytes per selection chunk, 8 per block when
 * block_norm2 is NULL and 8 x m x ceil(n / 2048) (dense; 8 x m for CSR) for
 * the partial products, each part rounded up to 256 bytes; larger problems
 * return RORBK_ERR_UNSUPPORTED before any device work.  Calls no hipMalloc,
 * hipFree or allocating routine.  Every call on a GPU shares that GPU's
 * array, which keeps the last call's contents: calls that overlap on one GPU
 * (other streams, other threads) race and must be serialised by the caller.
 * Blocks of more than RORBK_MAX_BIG_BLOCK_ROWS rows: RORBK_ERR_UNSUPPORTED. */
int ror_bk_residual_noalloc(const rorbk_matrix *A, int64_t block_rows, const void *b,
                            const void *x, void *r, double *block_norm2, double *rrn,
                            int32_t vec_f32, void *stream);

/* What the last solve on the handle recorded of Algorithm 1 (host buffers,
 * caller-owned, each may be NULL): tau (3*iters int32, the inner loop's
 * sampled blocks), the greedy sets I (iters*K int32, rows ascending; only
 * when the last solve ran with RECORD or CHECKPOINT, else
 * RORBK_ERR_NOT_RECORDED), and the history of the stop test's
 * RRN (iters doubles); *iters_host receives the iteration count.  A later
 * solve (of any kind) replaces the record.  Synchronises the stream. */
int ror_bk_get_record(rorbk_handle h, int32_t *tau_host, int32_t *I_host,
                      double *rrn_host, int64_t *iters_host);

/* The selections Algorithm 1 would otherwise make (the inner loop's three
 * sampled blocks and the greedy step's rows) for RORBK_REPLAY solves of up to
 * `iters` iterations: tau (3*iters int32, block indices in [0,k)), greedy sets
 * (iters*K int32, row indices in [0,m), strictly ascending within a set),
 * host memory, copied to the handle (device buffers allocated here).
 * RORBK_ERR_INVALID_ARG on an index out of range or a set out of order. */
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

/* Refinement controls for RORBK_REFINE (not in the paper: FP32/BF16 inner
 * passes of Algorithm 1 corrected by an FP64 outer residual): inner iterations
 * per FP64 correction (default 50) and the inner relative stop eta (default
 * 1e-4; the inner solve also stops once its residual is below tol * ||b||).
 * RORBK_ERR_INVALID_ARG if inner_iters < 1 or eta is negative or not finite. */
int ror_bk_set_refine(rorbk_handle h, int64_t inner_iters, double eta);

/* Timings of the full residual pass (Algorithm 1's r = b - A x, the O(mn)
 * part of every iteration, Section 3.1) in the last RORBK_PROFILE solve, into
 * out4_host (host, 4 doubles): out[0] = mean duration (ms) of the sampled
 * inner (working-precision) residual launches, out[1] = their count, out[2] =
 * mean duration (ms) of the FP64 outer residual launches of a REFINE solve,
 * out[3] = their count. */
int ror_bk_get_profile(rorbk_handle h, double *out4_host);

/* Static description of a status code (the RORBK_ERR_* list above; the
 * paper defines no error handling). */
const char *ror_bk_error_string(int code);

/* Details of the calling thread's last failure ("" if none); library
 * diagnostics, not a step of the method. */
const char *ror_bk_last_error_message(void);

#ifdef __cplusplus
}
#endif

#endif /* RORBK_H */
