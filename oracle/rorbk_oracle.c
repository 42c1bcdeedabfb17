/*
 * rorbk_oracle.c -- plain FP64 CPU oracle for ROR-BK
 * (Kar & Venkatapathi, "A fast solver for ill-conditioned linear systems using
 * randomized stable solutions of its blocks", arXiv 2510.02156).
 *
 * TEST INFRASTRUCTURE.  This is the slow, obviously-correct reference that the
 * HIP library is checked against.  Only the test suite, the package smoke check
 * and the benchmark's CPU-baseline leg may load it.  It shares no code, header
 * or table with the HIP library; both sides only see the same seeded inputs.
 *
 * Everything is FP64 in plain loops.  OpenMP parallelises outer loops whose
 * iterations are independent (rows of a residual, columns of an update, blocks
 * of the setup); every individual sum is still taken sequentially in index
 * order, so results do not depend on the thread count.
 *
 * Readings taken where the paper is silent (each is listed in the design notes):
 *  - the blocks: k = floor(m / block_rows) contiguous blocks; the first
 *    m - k*floor(m/k) blocks get one extra row ("at least floor(m/k) rows").
 *  - the sampler: inverse CDF over the FP64 prefix sums W of Pbar, driven by a
 *    counter-based SplitMix64 stream (word c = 3j + (l-1) of iteration j).
 *  - top-K: key |r_i|, ties to the lower index, indices returned ascending.
 *  - stop test: ||b - A x|| < tol * ||b||, strict, taken before the greedy step.
 *  - a zero centroid has C(t,t) = 1 and C(t,j) = 0 for j != t.
 * Parity pins for every function live in the test suite.
 */
#define _POSIX_C_SOURCE 199309L
#include <math.h>
#include <stdint.h>
#include <time.h>
#include <stdlib.h>
#include <string.h>

#define ORC_OK 0
#define ORC_ERR_ARG 1
#define ORC_ERR_OOM 2
#define ORC_ERR_NOT_SPD 4
#define ORC_ERR_NONFINITE 5

/* A dense row-major matrix (csr == 0: entry (i,j) = a[i*ld + j]) or CSR
 * (csr == 1: row i holds colidx/val[rowptr[i] .. rowptr[i+1]), columns sorted). */
typedef struct {
    int64_t m, n;
    int32_t csr;
    int32_t pad_;
    const double *a;
    int64_t ld;
    const int64_t *rowptr;
    const int32_t *colidx;
    const double *val;
} orc_matrix;

/* ------------------------------------------------------------------ rows -- */

/* <A_(i), x> summed in column order. */
static double row_dot(const orc_matrix *A, int64_t i, const double *x)
{
    double s = 0.0;
    if (!A->csr) {
        const double *ai = A->a + i * A->ld;
        for (int64_t j = 0; j < A->n; ++j) s += ai[j] * x[j];
    } else {
        for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
            s += A->val[p] * x[A->colidx[p]];
    }
    return s;
}

/* <A_(i), A_(j)>: dense in column order; CSR by merging the sorted rows. */
static double row_row_dot(const orc_matrix *A, int64_t i, int64_t j)
{
    double s = 0.0;
    if (!A->csr) {
        const double *ai = A->a + i * A->ld, *aj = A->a + j * A->ld;
        for (int64_t c = 0; c < A->n; ++c) s += ai[c] * aj[c];
    } else {
        int64_t p = A->rowptr[i], pe = A->rowptr[i + 1];
        int64_t q = A->rowptr[j], qe = A->rowptr[j + 1];
        while (p < pe && q < qe) {
            if (A->colidx[p] < A->colidx[q]) ++p;
            else if (A->colidx[p] > A->colidx[q]) ++q;
            else { s += A->val[p] * A->val[q]; ++p; ++q; }
        }
    }
    return s;
}

/* -------------------------------------------------------------- partition -- */

/* Number of blocks k for a requested block size (rows per block).
 * Algorithm 1 takes k blocks of at least floor(m/k) rows; the workloads give
 * rows per block, so k = floor(m / block_rows). */
int64_t orc_num_blocks(int64_t m, int64_t block_rows)
{
    if (m <= 0 || block_rows <= 0 || block_rows > m) return 0;
    return m / block_rows;
}

/* Algorithm 1, first step: contiguous aggregation of rows into k blocks, each
 * with at least floor(m/k) rows (Section 2).  The m - k*floor(m/k) leftover
 * rows go one each to the first blocks.  offsets has k+1 entries. */
void orc_partition(int64_t m, int64_t k, int64_t *offsets)
{
    int64_t q = m / k, rem = m - k * q;
    for (int64_t t = 0; t <= k; ++t)
        offsets[t] = t * q + (t < rem ? t : rem);
}

/* ------------------------------------------------------- orthogonality -- */

/* Section 2 and Algorithm 1 (second to fourth steps):
 *   centroid  Abar_t = sum of the rows of block t,
 *   C(i,j)    = |<Abar_i, Abar_j>| / (||Abar_i|| ||Abar_j||),
 *   S_t       = sum_{j=1..k} C(t,j)      (the diagonal term included),
 *   Pbar_t    = exp(-2 S_t / n),  P = Pbar / sum(Pbar),
 * and W_t = Pbar_0 + ... + Pbar_t, summed in order (the sampler's table).
 * Dense A keeps the centroids as a dense k x n matrix; CSR A keeps each
 * centroid as a sorted sparse row.  Only the rows t in [t_lo, t_hi) of S are
 * produced (the whole range for a full setup). */
typedef struct { int64_t nnz; int32_t *col; double *val; } sparse_vec;

static double sv_dot(const sparse_vec *a, const sparse_vec *b)
{
    double s = 0.0;
    int64_t p = 0, q = 0;
    while (p < a->nnz && q < b->nnz) {
        if (a->col[p] < b->col[q]) ++p;
        else if (a->col[p] > b->col[q]) ++q;
        else { s += a->val[p] * b->val[q]; ++p; ++q; }
    }
    return s;
}

int orc_cosine_rowsums(const orc_matrix *A, int64_t k, const int64_t *offsets,
                       int64_t t_lo, int64_t t_hi, double *S)
{
    const int64_t n = A->n;
    double *nrm = (double *)malloc(sizeof(double) * k);
    if (!nrm) return ORC_ERR_OOM;
    int rc = ORC_OK;
    if (!A->csr) {
        double *cen = (double *)calloc((size_t)(k * n), sizeof(double));
        if (!cen) { free(nrm); return ORC_ERR_OOM; }
        #pragma omp parallel for schedule(static)
        for (int64_t t = 0; t < k; ++t) {
            double *ct = cen + t * n;
            for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i) {
                const double *ai = A->a + i * A->ld;
                for (int64_t c = 0; c < n; ++c) ct[c] += ai[c];
            }
            double s = 0.0;
            for (int64_t c = 0; c < n; ++c) s += ct[c] * ct[c];
            nrm[t] = sqrt(s);
        }
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t t = t_lo; t < t_hi; ++t) {
            double acc = 0.0;
            for (int64_t j = 0; j < k; ++j) {
                double cij;
                if (nrm[t] == 0.0 || nrm[j] == 0.0) {
                    cij = (j == t) ? 1.0 : 0.0;
                } else {
                    double d = 0.0;
                    const double *ct = cen + t * n, *cj = cen + j * n;
                    for (int64_t c = 0; c < n; ++c) d += ct[c] * cj[c];
                    cij = fabs(d) / (nrm[t] * nrm[j]);
                }
                acc += cij;
            }
            S[t - t_lo] = acc;
        }
        free(cen);
    } else {
        sparse_vec *cen = (sparse_vec *)calloc((size_t)k, sizeof(sparse_vec));
        if (!cen) { free(nrm); return ORC_ERR_OOM; }
        int fail = 0;
        #pragma omp parallel
        {
            double *dense = (double *)calloc((size_t)n, sizeof(double));
            unsigned char *hit = (unsigned char *)calloc((size_t)n, 1);
            if (!dense || !hit) {
                #pragma omp atomic write
                fail = 1;
            }
            #pragma omp for schedule(dynamic, 4)
            for (int64_t t = 0; t < k; ++t) {
                if (fail) continue;
                /* accumulate the block's rows in row order, then list the
                 * touched columns in ascending order */
                for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
                    for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) {
                        dense[A->colidx[p]] += A->val[p];
                        hit[A->colidx[p]] = 1;
                    }
                int64_t cnt = 0;
                for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
                    cnt += A->rowptr[i + 1] - A->rowptr[i];
                int32_t *cols = (int32_t *)malloc(sizeof(int32_t) * (cnt ? cnt : 1));
                int64_t u = 0;
                for (int64_t i = offsets[t]; i < offsets[t + 1]; ++i)
                    for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p)
                        if (hit[A->colidx[p]] == 1) { hit[A->colidx[p]] = 2; cols[u++] = A->colidx[p]; }
                /* insertion sort keeps this obviously correct; blocks are small */
                for (int64_t a = 1; a < u; ++a) {
                    int32_t v = cols[a]; int64_t b = a - 1;
                    while (b >= 0 && cols[b] > v) { cols[b + 1] = cols[b]; --b; }
                    cols[b + 1] = v;
                }
                cen[t].nnz = u;
                cen[t].col = cols;
                cen[t].val = (double *)malloc(sizeof(double) * (u ? u : 1));
                double s = 0.0;
                for (int64_t a = 0; a < u; ++a) {
                    double v = dense[cols[a]];
                    cen[t].val[a] = v;
                    s += v * v;
                    dense[cols[a]] = 0.0;
                    hit[cols[a]] = 0;
                }
                nrm[t] = sqrt(s);
            }
            free(dense);
            free(hit);
        }
        if (fail) rc = ORC_ERR_OOM;
        if (rc == ORC_OK) {
            #pragma omp parallel for schedule(dynamic, 1)
            for (int64_t t = t_lo; t < t_hi; ++t) {
                double acc = 0.0;
                for (int64_t j = 0; j < k; ++j) {
                    double cij;
                    if (nrm[t] == 0.0 || nrm[j] == 0.0)
                        cij = (j == t) ? 1.0 : 0.0;
                    else
                        cij = fabs(sv_dot(&cen[t], &cen[j])) / (nrm[t] * nrm[j]);
                    acc += cij;
                }
                S[t - t_lo] = acc;
            }
        }
        for (int64_t t = 0; t < k; ++t) { free(cen[t].col); free(cen[t].val); }
        free(cen);
    }
    free(nrm);
    return rc;
}

/* Pbar_t = exp(-2 S_t / n) (Section 2, the proposal equation; Algorithm 1,
 * third step) and the running sums W used to sample P = Pbar / sum(Pbar). */
void orc_proposal(const double *S, int64_t k, int64_t n, double *pbar, double *W)
{
    double acc = 0.0;
    for (int64_t t = 0; t < k; ++t) {
        pbar[t] = exp(-2.0 * S[t] / (double)n);
        acc += pbar[t];
        W[t] = acc;
    }
}

/* ---------------------------------------------------------------- sampler -- */

/* SplitMix64 (Steele, Lea and Flood, OOPSLA 2014): the state advances by the
 * golden-ratio increment 0x9E3779B97F4A7C15 and each output is the state passed
 * through the 64-bit finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9,
 * xor-shift 27, multiply 0x94D049BB133111EB, xor-shift 31).  Used here as a
 * counter-based stream: word c of seed s is the finaliser applied to
 * s + (c + 1) * increment. */
uint64_t orc_splitmix64_word(uint64_t seed, uint64_t c)
{
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

/* Algorithm 1, inner loop: draw a block index from P = Pbar / sum(Pbar).
 * Draw l (1..3) of outer iteration j uses stream word c = 3j + (l - 1):
 * u = (word >> 11) * 2^-53 in [0,1), and tau is the number of prefix sums W_t
 * that do not exceed u * W_{k-1} (inverse CDF), clamped to k - 1. */
int32_t orc_sample(uint64_t seed, int64_t j, int32_t l, const double *W, int64_t k)
{
    uint64_t w = orc_splitmix64_word(seed, (uint64_t)(3 * j + (l - 1)));
    double u = (double)(w >> 11) * 0x1.0p-53;
    double target = u * W[k - 1];
    int64_t cnt = 0;
    for (int64_t t = 0; t < k; ++t)
        if (W[t] <= target) ++cnt;
    if (cnt > k - 1) cnt = k - 1;
    return (int32_t)cnt;
}

/* ------------------------------------------------------------ small solve -- */

/* In-place lower Cholesky G = L L^T of a dense K x K SPD matrix (row-major,
 * the lower triangle is read and overwritten).  Returns ORC_ERR_NOT_SPD on a
 * non-positive pivot. */
int orc_cholesky(double *G, int64_t K)
{
    for (int64_t j = 0; j < K; ++j) {
        double d = G[j * K + j];
        for (int64_t p = 0; p < j; ++p) d -= G[j * K + p] * G[j * K + p];
        if (!(d > 0.0)) return ORC_ERR_NOT_SPD;
        double ljj = sqrt(d);
        G[j * K + j] = ljj;
        for (int64_t i = j + 1; i < K; ++i) {
            double s = G[i * K + j];
            for (int64_t p = 0; p < j; ++p) s -= G[i * K + p] * G[j * K + p];
            G[i * K + j] = s / ljj;
        }
    }
    return ORC_OK;
}

/* y = (L L^T)^{-1} r by forward then backward substitution. */
void orc_chol_solve(const double *L, int64_t K, const double *r, double *y)
{
    for (int64_t i = 0; i < K; ++i) {
        double s = r[i];
        for (int64_t p = 0; p < i; ++p) s -= L[i * K + p] * y[p];
        y[i] = s / L[i * K + i];
    }
    for (int64_t i = K - 1; i >= 0; --i) {
        double s = y[i];
        for (int64_t p = i + 1; p < K; ++p) s -= L[p * K + i] * y[p];
        y[i] = s / L[i * K + i];
    }
}

/* G = A_S A_S^T + mu I for the rows S (K of them), then its Cholesky factor.
 * The regularised block operator of Algorithm 1; Section 3.1 stores the
 * factorisation of each fixed block once. */
int orc_block_factor(const orc_matrix *A, const int64_t *rows, int64_t K,
                     double mu, double *L)
{
    for (int64_t p = 0; p < K; ++p)
        for (int64_t q = 0; q <= p; ++q) {
            double g = row_row_dot(A, rows[p], rows[q]);
            if (p == q) g += mu;
            L[p * K + q] = g;
            L[q * K + p] = g;
        }
    return orc_cholesky(L, K);
}

/* One regularised block update (Lemma 2's update rule; Algorithm 1):
 *   x <- x + A_S^T (A_S A_S^T + mu I)^{-1} (b_S - A_S x),
 * with the factor L of A_S A_S^T + mu I given.  rS, if not NULL, supplies
 * b_S - A_S x already computed (the greedy step reuses the full residual).
 * ws needs K + K + n doubles. */
static void block_update(const orc_matrix *A, const int64_t *rows, int64_t K,
                         const double *L, const double *b, const double *rS,
                         double *x, double *ws)
{
    double *r = ws, *y = ws + K, *u = ws + 2 * K;
    for (int64_t p = 0; p < K; ++p)
        r[p] = rS ? rS[p] : b[rows[p]] - row_dot(A, rows[p], x);
    orc_chol_solve(L, K, r, y);
    /* u = A_S^T y, summed over the rows of S in order; then x += u */
    const int64_t n = A->n;
    if (!A->csr) {
        #pragma omp parallel for schedule(static)
        for (int64_t c = 0; c < n; ++c) {
            double s = 0.0;
            for (int64_t p = 0; p < K; ++p) s += A->a[rows[p] * A->ld + c] * y[p];
            u[c] = s;
        }
    } else {
        for (int64_t c = 0; c < n; ++c) u[c] = 0.0;
        for (int64_t p = 0; p < K; ++p)
            for (int64_t q = A->rowptr[rows[p]]; q < A->rowptr[rows[p] + 1]; ++q)
                u[A->colidx[q]] += A->val[q] * y[p];
    }
    #pragma omp parallel for schedule(static)
    for (int64_t c = 0; c < n; ++c) x[c] += u[c];
}

/* A single regularised block update on the rows S (factor formed here):
 * x <- x + A_S^T (A_S A_S^T + mu I)^{-1} (b_S - A_S x).  For tests of the
 * update's identities (Lemma 1, Theorem 1's error relation). */
int orc_apply_block(const orc_matrix *A, const int64_t *rows, int64_t K,
                    double mu, const double *b, double *x)
{
    double *L = (double *)malloc(sizeof(double) * K * K);
    double *ws = (double *)malloc(sizeof(double) * (2 * K + A->n));
    int rc = (L && ws) ? ORC_OK : ORC_ERR_OOM;
    if (rc == ORC_OK) rc = orc_block_factor(A, rows, K, mu, L);
    if (rc == ORC_OK) block_update(A, rows, K, L, b, NULL, x, ws);
    free(L);
    free(ws);
    return rc;
}

/* ---------------------------------------------------------- residual, top-K */

/* r = b - A x  (Algorithm 1, after the three sampled updates). */
void orc_residual(const orc_matrix *A, const double *b, const double *x, double *r)
{
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < A->m; ++i) r[i] = b[i] - row_dot(A, i, x);
}

static const double *g_topk_key;
static int topk_cmp(const void *pa, const void *pb)
{
    int64_t a = *(const int64_t *)pa, b = *(const int64_t *)pb;
    double ka = fabs(g_topk_key[a]), kb = fabs(g_topk_key[b]);
    if (ka > kb) return -1;
    if (ka < kb) return 1;
    return (a < b) ? -1 : (a > b);
}
static int idx_cmp(const void *pa, const void *pb)
{
    int32_t a = *(const int32_t *)pa, b = *(const int32_t *)pb;
    return (a > b) - (a < b);
}

/* Algorithm 1, greedy step: the indices of the K largest r_i^2 (ordered by
 * |r_i|, which orders r_i^2 without rounding the square; ties go to the lower
 * index), returned in ascending order.  ORC_ERR_NONFINITE on a NaN. */
int orc_topk(const double *r, int64_t m, int64_t K, int32_t *idx)
{
    for (int64_t i = 0; i < m; ++i)
        if (isnan(r[i])) return ORC_ERR_NONFINITE;
    int64_t *ord = (int64_t *)malloc(sizeof(int64_t) * m);
    if (!ord) return ORC_ERR_OOM;
    for (int64_t i = 0; i < m; ++i) ord[i] = i;
    g_topk_key = r;
    qsort(ord, (size_t)m, sizeof(int64_t), topk_cmp);
    for (int64_t p = 0; p < K; ++p) idx[p] = (int32_t)ord[p];
    qsort(idx, (size_t)K, sizeof(int32_t), idx_cmp);
    free(ord);
    return ORC_OK;
}

/* ------------------------------------------------------------------ solve -- */

/* Algorithm 1.  Iterations j = start_iter .. start_iter + max_iters - 1:
 *   three sampled regularised updates (tau drawn from P),
 *   r = b - A x and the stop test ||r|| < tol ||b||  (return before the greedy
 *   step when it holds),
 *   the greedy update on the rows I of the K = floor(m/k) largest |r_i|,
 *   using r_I from the residual just computed (x has not moved since).
 * Setup: partition, proposal, and the factor of every fixed block.
 * replay_tau / replay_I (NULL = free running) inject the selections;
 * rec_tau, rec_I, rec_rrn (NULL = off) receive them, indexed from start_iter.
 * W_in, if not NULL, replaces the proposal table (k entries).
 * out_ints = {iterations run, converged}; out_rrn = last measured RRN;
 * out_times (NULL = off) = {setup seconds, iteration seconds} (wall clock). */
static double now_s(void)
{
    struct timespec ts;
    clock_gettime(CLOCK_MONOTONIC, &ts);
    return (double)ts.tv_sec + 1e-9 * (double)ts.tv_nsec;
}

int orc_solve(const orc_matrix *A, int64_t block_rows, double mu,
              const double *b, double *x, uint64_t seed, double tol,
              int64_t max_iters, int64_t start_iter,
              const double *W_in,
              const int32_t *replay_tau, const int32_t *replay_I,
              int32_t *rec_tau, int32_t *rec_I, double *rec_rrn,
              int64_t *out_ints, double *out_rrn, double *out_times)
{
    const double t_start = now_s();
    double t_iter = 0.0;
    const int64_t m = A->m, n = A->n;
    int64_t k = orc_num_blocks(m, block_rows);
    if (k <= 0 || mu < 0.0) return ORC_ERR_ARG;
    const int64_t K = m / k;
    int rc = ORC_OK;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
    double *S = (double *)malloc(sizeof(double) * k);
    double *pbar = (double *)malloc(sizeof(double) * k);
    double *W = (double *)malloc(sizeof(double) * k);
    double **Lt = (double **)calloc((size_t)k, sizeof(double *));
    double *r = (double *)malloc(sizeof(double) * m);
    double *ws = (double *)malloc(sizeof(double) * (2 * (K + 1) + n));
    double *LI = (double *)malloc(sizeof(double) * K * K);
    double *rI = (double *)malloc(sizeof(double) * K);
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (K + 1));
    int32_t *I = (int32_t *)malloc(sizeof(int32_t) * K);
    if (!off || !S || !pbar || !W || !Lt || !r || !ws || !LI || !rI || !rows || !I) {
        rc = ORC_ERR_OOM;
        goto done;
    }
    orc_partition(m, k, off);
    if (W_in) {
        memcpy(W, W_in, sizeof(double) * k);
    } else {
        rc = orc_cosine_rowsums(A, k, off, 0, k, S);
        if (rc) goto done;
        orc_proposal(S, k, n, pbar, W);
    }
    /* factor every fixed block once (Section 3.1) */
    {
        int bad = 0;
        #pragma omp parallel for schedule(dynamic, 1)
        for (int64_t t = 0; t < k; ++t) {
            int64_t bt = off[t + 1] - off[t];
            int64_t *rr = (int64_t *)malloc(sizeof(int64_t) * bt);
            Lt[t] = (double *)malloc(sizeof(double) * bt * bt);
            if (!rr || !Lt[t]) { bad = ORC_ERR_OOM; free(rr); continue; }
            for (int64_t p = 0; p < bt; ++p) rr[p] = off[t] + p;
            if (orc_block_factor(A, rr, bt, mu, Lt[t]) != ORC_OK) bad = ORC_ERR_NOT_SPD;
            free(rr);
        }
        if (bad) { rc = bad; goto done; }
    }
    double bnorm2 = 0.0;
    for (int64_t i = 0; i < m; ++i) bnorm2 += b[i] * b[i];
    const double thresh = tol * sqrt(bnorm2);
    t_iter = now_s();
    int64_t it = 0;
    int converged = 0;
    double rrn = NAN;
    for (; it < max_iters; ++it) {
        const int64_t j = start_iter + it;
        for (int32_t l = 1; l <= 3; ++l) {
            int32_t tau = replay_tau ? replay_tau[3 * it + (l - 1)]
                                     : orc_sample(seed, j, l, W, k);
            if (tau < 0 || tau >= k) { rc = ORC_ERR_ARG; goto done; }
            if (rec_tau) rec_tau[3 * it + (l - 1)] = tau;
            int64_t bt = off[tau + 1] - off[tau];
            for (int64_t p = 0; p < bt; ++p) rows[p] = off[tau] + p;
            block_update(A, rows, bt, Lt[tau], b, NULL, x, ws);
        }
        orc_residual(A, b, x, r);
        double rn2 = 0.0;
        for (int64_t i = 0; i < m; ++i) rn2 += r[i] * r[i];
        if (!isfinite(rn2)) { rc = ORC_ERR_NONFINITE; goto done; }
        double rn = sqrt(rn2);
        rrn = (bnorm2 > 0.0) ? rn / sqrt(bnorm2) : 0.0;
        if (rec_rrn) rec_rrn[it] = rrn;
        if (rn < thresh) { converged = 1; ++it; break; }
        if (replay_I) {
            memcpy(I, replay_I + it * K, sizeof(int32_t) * K);
        } else {
            rc = orc_topk(r, m, K, I);
            if (rc) goto done;
        }
        if (rec_I) memcpy(rec_I + it * K, I, sizeof(int32_t) * K);
        for (int64_t p = 0; p < K; ++p) {
            if (I[p] < 0 || I[p] >= m) { rc = ORC_ERR_ARG; goto done; }
            rows[p] = I[p];
            rI[p] = r[I[p]];
        }
        if (orc_block_factor(A, rows, K, mu, LI) != ORC_OK) { rc = ORC_ERR_NOT_SPD; goto done; }
        block_update(A, rows, K, LI, b, rI, x, ws);
    }
    if (out_ints) { out_ints[0] = it; out_ints[1] = converged; }
    if (out_rrn) *out_rrn = rrn;
    if (out_times) {
        const double t_end = now_s();
        out_times[0] = t_iter - t_start;
        out_times[1] = t_end - t_iter;
    }
done:
    if (Lt) for (int64_t t = 0; t < k; ++t) free(Lt[t]);
    free(off); free(S); free(pbar); free(W); free(Lt); free(r); free(ws);
    free(LI); free(rI); free(rows); free(I);
    return rc;
}

/* ---------------------------------------------------------------- adjoint -- */

/* Reverse-mode derivative of the recorded iteration.  With the selections held
 * fixed, every step x' = x + A_S^T H_S (b_S - A_S x), H_S = (A_S A_S^T + mu I)^{-1}
 * (the update rule of Lemma 2) is linear in (x, b), so for a cotangent g' of x'
 *   y = H_S A_S g',   gb[S] += y,   g = g' - A_S^T y.
 * Steps are undone newest first; an iteration contributes its three sampled
 * steps and, unless it was the converged one, its greedy step.  On entry g
 * holds dL/dx_final; on return gb = dL/db and g = dL/dx0. */
int orc_backward(const orc_matrix *A, int64_t block_rows, double mu,
                 const int32_t *tau, const int32_t *Isets, int64_t iters,
                 int32_t last_converged, double *g, double *gb)
{
    const int64_t m = A->m, n = A->n;
    int64_t k = orc_num_blocks(m, block_rows);
    if (k <= 0) return ORC_ERR_ARG;
    const int64_t K = m / k;
    int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (k + 1));
    int64_t *rows = (int64_t *)malloc(sizeof(int64_t) * (K + 1));
    double *L = (double *)malloc(sizeof(double) * (K + 1) * (K + 1));
    double *v = (double *)malloc(sizeof(double) * (K + 1));
    double *y = (double *)malloc(sizeof(double) * (K + 1));
    double *u = (double *)malloc(sizeof(double) * n);
    int rc = ORC_OK;
    if (!off || !rows || !L || !v || !y || !u) { rc = ORC_ERR_OOM; goto done; }
    orc_partition(m, k, off);
    for (int64_t i = 0; i < m; ++i) gb[i] = 0.0;
    for (int64_t it = iters - 1; it >= 0; --it) {
        int has_greedy = !(it == iters - 1 && last_converged);
        for (int step = has_greedy ? 3 : 2; step >= 0; --step) {
            int64_t KS;
            if (step == 3) {
                KS = K;
                for (int64_t p = 0; p < K; ++p) rows[p] = Isets[it * K + p];
            } else {
                int32_t t = tau[3 * it + step];
                KS = off[t + 1] - off[t];
                for (int64_t p = 0; p < KS; ++p) rows[p] = off[t] + p;
            }
            if (orc_block_factor(A, rows, KS, mu, L) != ORC_OK) { rc = ORC_ERR_NOT_SPD; goto done; }
            for (int64_t p = 0; p < KS; ++p) v[p] = row_dot(A, rows[p], g);
            orc_chol_solve(L, KS, v, y);
            for (int64_t p = 0; p < KS; ++p) gb[rows[p]] += y[p];
            for (int64_t c = 0; c < n; ++c) u[c] = 0.0;
            if (!A->csr) {
                for (int64_t p = 0; p < KS; ++p) {
                    const double *ar = A->a + rows[p] * A->ld;
                    for (int64_t c = 0; c < n; ++c) u[c] += ar[c] * y[p];
                }
            } else {
                for (int64_t p = 0; p < KS; ++p)
                    for (int64_t q = A->rowptr[rows[p]]; q < A->rowptr[rows[p] + 1]; ++q)
                        u[A->colidx[q]] += A->val[q] * y[p];
            }
            for (int64_t c = 0; c < n; ++c) g[c] -= u[c];
        }
    }
done:
    free(off); free(rows); free(L); free(v); free(y); free(u);
    return rc;
}

/* ------------------------------------------------- initial solution (App.) */

/* Algorithm 2 of the appendix (initial solution): y = the sum of all rows of
 * A (each entry summed over the rows in ascending row order), b~ = A y, and
 * x0 = (<b, b~> / ||b~||^2) y.  The remark after Algorithm 2: x0 lies in the
 * row space of A and ||b - A x0|| <= ||b||.  When b~ = 0 the coefficient is 0
 * (x0 = 0).  *alpha receives the coefficient. */
int orc_initial_solution(const orc_matrix *A, const double *b, double *x0, double *alpha)
{
    const int64_t m = A->m, n = A->n;
    double *y = (double *)calloc((size_t)n, sizeof(double));
    double *bt = (double *)malloc(sizeof(double) * (size_t)m);
    if (!y || !bt) { free(y); free(bt); return ORC_ERR_OOM; }
    for (int64_t i = 0; i < m; ++i) {
        if (!A->csr) {
            const double *ai = A->a + i * A->ld;
            for (int64_t c = 0; c < n; ++c) y[c] += ai[c];
        } else {
            for (int64_t p = A->rowptr[i]; p < A->rowptr[i + 1]; ++p) y[A->colidx[p]] += A->val[p];
        }
    }
    #pragma omp parallel for schedule(static)
    for (int64_t i = 0; i < m; ++i) bt[i] = row_dot(A, i, y);
    double bb = 0.0, tt = 0.0;
    for (int64_t i = 0; i < m; ++i) {
        bb += b[i] * bt[i];
        tt += bt[i] * bt[i];
    }
    const double a = (tt > 0.0) ? bb / tt : 0.0;
    for (int64_t c = 0; c < n; ++c) x0[c] = a * y[c];
    if (alpha) *alpha = a;
    free(y);
    free(bt);
    return ORC_OK;
}

/* ------------------------------------ flexible AB-GMRES (App., Algorithm 3) */

/* Algorithm 3 of the appendix: flexible AB-GMRES with ROR-BK as the right
 * preconditioner.  From x (x0 in, result out): r0 = b - A x0, beta = ||r0||,
 * v_1 = r0 / beta.  Outer step k: z_k = ROR-BK (Algorithm 1) on A z = v_k from
 * z = 0 for at most inner_iters iterations, stopping once ||v_k - A z|| <
 * eta ||v_k||; its sampler counter starts at (k - 1) * inner_iters, so every
 * outer step draws fresh blocks from the same stream.  w = A z_k is
 * orthogonalised against v_1..v_k by modified Gram-Schmidt (h_ik = <w, v_i>,
 * w -= h_ik v_i), h_{k+1,k} = ||w||, v_{k+1} = w / h_{k+1,k}.  The Hessenberg
 * least-squares problem min ||beta e_1 - H y|| is kept reduced with Givens
 * rotations; the outer loop stops when its residual |g_{k+1}| < tol ||b||,
 * when h_{k+1,k} = 0, or after max_outer steps.  Then x = x0 + Z y.
 * W: the sampler's running sums (NULL: computed here).  Outputs: *outer
 * steps taken, res_hist[k] = |g_{k+1}| / ||b|| per step, and (optional) Z
 * (n x max_outer, column k at Z + k n) and H ((max_outer + 1) x max_outer,
 * column-major, before the rotations). */
int orc_fabgmres(const orc_matrix *A, int64_t block_rows, double mu, const double *b,
                 double *x, uint64_t seed, double tol, int64_t max_outer, int64_t inner_iters,
                 double eta, const double *W_in, int64_t *outer, double *res_hist, double *Zout,
                 double *Hout)
{
    const int64_t m = A->m, n = A->n;
    const int64_t kb = orc_num_blocks(m, block_rows);
    if (kb <= 0 || max_outer < 1 || inner_iters < 1) return ORC_ERR_ARG;
    const int64_t M1 = max_outer + 1;
    double *V = (double *)malloc(sizeof(double) * (size_t)(m * M1));
    double *Z = (double *)calloc((size_t)(n * max_outer), sizeof(double));
    double *H = (double *)calloc((size_t)(M1 * max_outer), sizeof(double));
    double *R = (double *)calloc((size_t)(M1 * max_outer), sizeof(double));
    double *cs = (double *)malloc(sizeof(double) * (size_t)max_outer);
    double *sn = (double *)malloc(sizeof(double) * (size_t)max_outer);
    double *g = (double *)calloc((size_t)M1, sizeof(double));
    double *w = (double *)malloc(sizeof(double) * (size_t)m);
    double *W = (double *)malloc(sizeof(double) * (size_t)kb);
    double *yv = (double *)calloc((size_t)max_outer, sizeof(double));
    int rc = ORC_OK;
    if (!V || !Z || !H || !R || !cs || !sn || !g || !w || !W || !yv) { rc = ORC_ERR_OOM; goto done; }
    if (W_in) {
        memcpy(W, W_in, sizeof(double) * (size_t)kb);
    } else {
        int64_t *off = (int64_t *)malloc(sizeof(int64_t) * (size_t)(kb + 1));
        double *S = (double *)malloc(sizeof(double) * (size_t)kb);
        double *pb = (double *)malloc(sizeof(double) * (size_t)kb);
        if (!off || !S || !pb) { free(off); free(S); free(pb); rc = ORC_ERR_OOM; goto done; }
        orc_partition(m, kb, off);
        rc = orc_cosine_rowsums(A, kb, off, 0, kb, S);
        if (!rc) orc_proposal(S, kb, n, pb, W);
        free(off); free(S); free(pb);
        if (rc) goto done;
    }
    double bn = 0.0;
    for (int64_t i = 0; i < m; ++i) bn += b[i] * b[i];
    bn = sqrt(bn);
    orc_residual(A, b, x, w);
    double beta = 0.0;
    for (int64_t i = 0; i < m; ++i) beta += w[i] * w[i];
    beta = sqrt(beta);
    *outer = 0;
    if (beta == 0.0) goto done;
    for (int64_t i = 0; i < m; ++i) V[i] = w[i] / beta;
    g[0] = beta;
    int64_t kend = 0;
    for (int64_t k = 0; k < max_outer; ++k) {
        /* z_k: inner ROR-BK on A z = v_k from zero */
        double *zk = Z + k * n;
        int64_t ints[2];
        double rrn, times[2];
        rc = orc_solve(A, block_rows, mu, V + k * m, zk, seed, eta, inner_iters,
                       k * inner_iters, W, NULL, NULL, NULL, NULL, NULL, ints, &rrn, times);
        if (rc) goto done;
        /* w = A z_k, modified Gram-Schmidt against v_1..v_k */
        #pragma omp parallel for schedule(static)
        for (int64_t i = 0; i < m; ++i) w[i] = row_dot(A, i, zk);
        for (int64_t i2 = 0; i2 <= k; ++i2) {
            const double *vi = V + i2 * m;
            double h = 0.0;
            for (int64_t i = 0; i < m; ++i) h += w[i] * vi[i];
            for (int64_t i = 0; i < m; ++i) w[i] -= h * vi[i];
            H[k * M1 + i2] = h;
        }
        double hn = 0.0;
        for (int64_t i = 0; i < m; ++i) hn += w[i] * w[i];
        hn = sqrt(hn);
        H[k * M1 + k + 1] = hn;
        if (hn > 0.0)
            for (int64_t i = 0; i < m; ++i) V[(k + 1) * m + i] = w[i] / hn;
        /* Givens: earlier rotations on column k, then a new one */
        for (int64_t i2 = 0; i2 <= k + 1; ++i2) R[k * M1 + i2] = H[k * M1 + i2];
        for (int64_t i2 = 0; i2 < k; ++i2) {
            const double a = R[k * M1 + i2], c = R[k * M1 + i2 + 1];
            R[k * M1 + i2] = cs[i2] * a + sn[i2] * c;
            R[k * M1 + i2 + 1] = -sn[i2] * a + cs[i2] * c;
        }
        const double a = R[k * M1 + k], c = R[k * M1 + k + 1];
        const double d = sqrt(a * a + c * c);
        cs[k] = (d > 0.0) ? a / d : 1.0;
        sn[k] = (d > 0.0) ? c / d : 0.0;
        R[k * M1 + k] = d;
        R[k * M1 + k + 1] = 0.0;
        g[k + 1] = -sn[k] * g[k];
        g[k] = cs[k] * g[k];
        if (res_hist) res_hist[k] = fabs(g[k + 1]) / (bn > 0.0 ? bn : 1.0);
        kend = k + 1;
        if (fabs(g[k + 1]) < tol * bn || hn == 0.0) break;
    }
    /* R y = g (upper triangular), x = x0 + Z y */
    for (int64_t i2 = kend - 1; i2 >= 0; --i2) {
        double s2 = g[i2];
        for (int64_t j = i2 + 1; j < kend; ++j) s2 -= R[j * M1 + i2] * yv[j];
        yv[i2] = s2 / R[i2 * M1 + i2];
    }
    for (int64_t j = 0; j < kend; ++j)
        for (int64_t c2 = 0; c2 < n; ++c2) x[c2] += yv[j] * Z[j * n + c2];
    *outer = kend;
    if (Zout) memcpy(Zout, Z, sizeof(double) * (size_t)(n * max_outer));
    if (Hout) memcpy(Hout, H, sizeof(double) * (size_t)(M1 * max_outer));
done:
    free(V); free(Z); free(H); free(R); free(cs); free(sn); free(g); free(w); free(W); free(yv);
    return rc;
}

/* Number of threads OpenMP will use (reported with the CPU timings), and a
 * way to change it for a timing run (results never depend on it: every sum
 * is sequential in index order). */
#ifdef _OPENMP
#include <omp.h>
int orc_num_threads(void) { return omp_get_max_threads(); }
void orc_set_num_threads(int t) { if (t > 0) omp_set_num_threads(t); }
#else
int orc_num_threads(void) { return 1; }
void orc_set_num_threads(int t) { (void)t; }
#endif
