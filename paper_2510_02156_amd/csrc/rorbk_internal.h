// rorbk_internal.h -- handle layout and kernel launchers of the MI355X ROR-BK
// library.  Internal to the library; the public ABI is include/rorbk.h.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "../../include/rorbk.h"

namespace rorbk {

// The greedy Gram of a large greedy set (dense, more than 161 rows) runs on
// 64 x 64 tiles for FP64 storage with at least this many rows, else on
// 32 x 32 tiles.
constexpr int GRAM64_MIN_K = 256;
__host__ __device__ constexpr bool gram64_for(int32_t dtype, int64_t K) {
    return dtype == RORBK_F64 && K >= GRAM64_MIN_K;
}

// Device-resident control block.  Written only by the single-workgroup
// selection and solve kernels; every iteration kernel reads `done` first and
// returns at once when it is set (the stop test, Algorithm 1, ends the solve
// before the greedy step).
struct Ctrl {
    int32_t done;        // 1 once converged or failed
    int32_t status;      // RORBK_OK, RORBK_ERR_NONFINITE or RORBK_ERR_NOT_SPD
    int64_t conv_it;     // iteration index (from the solve's start) that stopped
    double bnorm2;       // ||b||^2 of the current right-hand side
    double thr;          // stop when ||r|| < thr (tol * ||b||)
    double rnorm2;       // last measured ||r||^2
    int64_t last_it;     // last iteration whose residual was measured
    double pad[2];
};

// Blocks of at most this many rows (dense, row form) run the fused forward
// steps of k_fwd.hip: the three sampled updates in one launch.
constexpr int RORBK_FWD_MAX_BLOCK = 65;

// The cross-Gram tile jobs a residual launch carries (jobs == 0: none).
struct XgSide {
    const int32_t *tau;
    int64_t ti;            // index of the iteration's first draw
    int64_t q, rem;
    int bmax;
    int jobs;
    double *out;           // [3][bmax][bmax]
};

// Vector-type tag: double (FP64 solve) or float (FP32/BF16 storage solve).
enum VecType { VEC_F64 = 0, VEC_F32 = 1 };

// Row set of one block step: a fixed block (its index read on the device from
// tau[tau_index]) or a gathered set of `count` rows at `idx`.
struct RowSel {
    int32_t kind;         // 0 fixed block via tau, 1 gathered, -1 none
    int32_t count;        // gathered: number of rows
    int64_t tau_index;    // fixed: index into the tau array
    const int32_t *idx;   // gathered: row indices (device)
};

struct Layout {
    int64_t m, n, ld, nnz;
    int32_t format, dtype;
    int64_t k, q, rem, K, bmax;
    // update kernel column chunks
    int64_t wu;           // columns per update workgroup (multiple of 128)
    int32_t nch_u;        // update chunks
    // greedy Gram column chunks
    int64_t wg;           // columns per Gram workgroup
    int32_t nch_g;
    // residual segments (2048 columns each)
    int32_t nseg;
    // selection chunks (whole blocks)
    int64_t bpc;          // blocks per selection chunk
    int32_t nch_s;        // selection chunks
    int32_t nch_f;        // fused forward steps: column slabs
    int64_t wf;           //   columns per slab (sub-slabs of 64 (FP64) or 128 columns)
    int32_t nch_c;        // chain form: column chunks of the Grams after the selection
    int64_t wc;           //   columns per chunk (a multiple of 32)
};

}  // namespace rorbk

struct rorbk_handle_s {
    rorbk::Layout L;
    hipStream_t stream;
    int32_t ncu;              // compute units of the device
    double lambda;
    double t_setup_s;         // wall time of ror_bk_setup
    int32_t aligned;          // 16-byte vector loads allowed on the matrix
    int32_t aligned64;        // same for the FP64 master copy
    const void *A;            // working matrix values (non-owning)
    const double *A64;        // FP64 master (non-owning, may be NULL)
    const int64_t *rowptr;    // CSR (non-owning)
    const int32_t *colidx;

    // setup results (owned)
    int64_t *d_off;           // k+1
    double *d_S, *d_pbar, *d_W;
    int64_t *d_hoff;          // k+1 offsets into d_H
    double *d_H;              // stored block inverses
    // per-solve workspaces (owned)
    rorbk::Ctrl *d_ctrl;
    rorbk::Ctrl *h_ctrl;      // pinned mirror
    uint32_t *d_selcnt;       // selection workgroups done (fused merge), 0 between launches
    double *d_ysum;           // sum of the rows of A (n), for the initial solution
    float *d_ysum32;          // the same in FP32 (allocated on first use)
    double *d_alg2;           // <b, A y>, ||A y||^2, coefficient
    // large-block path (dense blocks of more than RORBK_MAX_BLOCK_ROWS + 1 rows)
    int32_t big;              // 1 when the large-block kernels run the steps
    int32_t col;              // 1: column form (blocks with at least as many rows as
                              // columns): n x n stored inverses and greedy system
    double *d_bigG;           // greedy system, padded, with the right-hand-side row
    double *d_bigL;           // its Cholesky factor (same layout)
    double *d_bigW;           // inverses of its diagonal tiles
    double *d_bigr;           // r_S of a fixed block step (bmax)
    double *d_bigy;           // y of a fixed block step (bmax)
    void *d_xold;             // x before the step's update (vector type, n)
    void *d_dxp;              // update column partials [row chunk][n] (vector type)
    double *d_P[2];           // partial A_S x per update chunk [nch][bmax]
    int32_t fast3;            // 1: fused forward steps (k_fwd.hip)
    double *d_P3;             // fused path: partial products of three blocks [nch][3 bmax]
    double *d_XG;             // fused path: cross-Grams, two slots [2][3][bmax][bmax]
    double *d_z3;             // fused path: z = b_S - A_S x of the next three blocks
    int32_t chain;            // chain form of the fused path (K <= 64, n <= 4096)
    double *d_C;              // chain form: A_{S'} A_I^T, [3 * FWD_B][64]
    uint32_t *d_fwdcnt;       // fused path: greedy workgroups done, 0 between launches
    double *d_axp;            // residual partial products [nseg][m]
    void *d_r;                // residual (vector type)
    double *d_bn;             // per-block ||r_t||^2
    double *d_cn;             // per-chunk ||r||^2
    uint64_t *d_ckey;         // selection candidates: keys
    int32_t *d_cidx;          //                        indices
    uint64_t *d_ckey2;        // second level of candidates
    int32_t *d_cidx2;
    int32_t *d_I;             // current greedy set (K)
    double *d_rI;             // r on the greedy set (K)
    double *d_y;              // greedy step solution (K)
    double *d_G;              // Gram partials [nch_g][K*K]
    double *d_red;            // scratch for norms
    int32_t *d_tau;           // block draws of the current solve (3 * cap)
    int64_t tau_cap;
    // refinement
    void *d_rhs32;            // float right-hand side of the inner solve
    void *d_d32;              // float correction
    double *d_r64;            // FP64 outer residual
    int64_t refine_inner;
    double refine_eta;
    // records
    int32_t *d_recI;          // greedy sets [cap][K]
    double *d_recR;           // RRN history [cap]
    int64_t rec_cap;
    int64_t rec_iters;        // iterations recorded by the last solve
    int32_t rec_valid;        // 1 after a RECORD solve, 2 after CHECKPOINT
    int32_t rec_I_valid;      // 1 while d_recI holds the greedy sets of the last solve
    int32_t rec_converged;
    int64_t ckpt_every;
    void *d_ckpt;             // x checkpoints (vector type) [(cap/c)+1][n]
    int64_t ckpt_cap;
    double *d_ckst;           // chain form: the rest of each checkpoint's state
                              // [slots][CKST_DOUBLES] (greedy rows, y, next z)
    int64_t ckst_cap;
    const void *rec_b;        // b of the recorded solve (CHECKPOINT recompute)
    uint64_t rec_seed;
    int32_t rec_vec;          // vector type of the recorded solve
    double rec_thr;           // stop threshold of the recorded solve
    // replay
    int32_t *d_rep_tau;
    int32_t *d_rep_I;
    int64_t rep_iters;
    // events
    hipEvent_t ev0, ev1;
    hipEvent_t evr[2][2];     // residual timing (start, end) per poll slot
    int32_t profile;
    double prof_in_ms, prof_out_ms;
    int64_t prof_in_n, prof_out_n;
};

namespace rorbk {

// ---------------------------------------------------------------- launchers
// Each returns hipSuccess or the launch error.  `vec` is VecType; `dt` is the
// storage dtype of the matrix pointer passed.

hipError_t launch_partition(int64_t m, int64_t k, int64_t *off, int64_t *hoff,
                            hipStream_t s);

hipError_t launch_sample(uint64_t seed, int64_t j0, int64_t count,
                         const double *W, int64_t k, int32_t *tau, hipStream_t s);

hipError_t launch_norm2(const void *v, int vec, int64_t len, double *red,
                        double *out, hipStream_t s);

hipError_t launch_copy_tau(const int32_t *src, int32_t *dst, int64_t count,
                           hipStream_t s);

// dense setup
hipError_t launch_setup_proposal_dense(const rorbk_handle_s *h, const void *A,
                                       int dt, int aligned, double *scratch,
                                       hipStream_t s);
hipError_t launch_block_inverses_dense(const rorbk_handle_s *h, const void *A,
                                       int dt, int aligned, int32_t *d_fail,
                                       hipStream_t s);
// doubles of device scratch the proposal setup needs (centroids, norms, row
// sums, centroid Gram parts)
int64_t setup_proposal_scratch(int64_t k, int64_t n, int ncu);
hipError_t launch_proposal_from_centroids(const rorbk_handle_s *h, double *cen, double *nrm,
                                          double *Sp, hipStream_t s);
// stored inverses (G_t + lambda I)^{-1} from packed block Grams Gs[t][kp]
hipError_t launch_block_inverses_from_grams(const rorbk_handle_s *h, const double *Gs,
                                            int64_t kp, int32_t *d_fail, hipStream_t s);
// CSR setup (values of dtype dt with the handle's rowptr / colidx)
hipError_t launch_csr_check(const rorbk_handle_s *h, int32_t *bad, hipStream_t s);
hipError_t launch_setup_proposal_csr(const rorbk_handle_s *h, const void *vals, int dt,
                                     double *scratch, hipStream_t s);
hipError_t launch_block_inverses_csr(const rorbk_handle_s *h, const void *vals, int dt,
                                     int32_t *d_fail, hipStream_t s);
// iteration kernels (dense or CSR chosen from the handle's format)
struct StepArgs {
    const void *A;        // matrix values (dtype dt)
    int dt;
    int aligned;
    int vec;
    const void *b;        // right-hand side (vector type) or NULL (adjoint)
    void *x;              // iterate (vector type)
    void *gb;             // adjoint: dL/db accumulator (vector type) or NULL
    RowSel cur;           // step applied
    int ymode;            // 0: y from partials + stored inverse; 1: y given (column
                          // form: the correction dx given); 2: none; 3: y given,
                          // x += A_S^T y in either form (column-form adjoint)
    const double *Pin;    // partials of the current step
    const double *ygiven;
    RowSel nxt;           // rows whose partial products are produced
    double *Pout;
};

// selection: builds r = b - sum(axp), block norms, candidates; then the final
// merge writes I, r_I, the RRN record and the stop flag.
struct SelectArgs {
    int vec;
    const void *b;
    const double *axp;    // NULL: r = b exactly (top-K of a given vector)
    int nseg;
    void *r;
    int64_t it;           // iteration index for records
    int record_rrn;
    double *rec_rrn;
    int record_I;
    int32_t *rec_I;       // [it*K]
    const int32_t *replay_I; // NULL or [it*K]
    int32_t *I_out;
    double *rI_out;
    int stop_test;        // 1: compare with thr2 and set done
    int skip_topk;        // 1: only norms (refinement outer residual)
    // spare workgroups (may be unset): the cross-Grams of the blocks drawn at
    // tau[xg_ti .. xg_ti+2] into xg_out, computed alongside the selection
    double *xg_out;
    const void *xg_A;
    int xg_dt;
    int xg_aligned;
    int64_t xg_ti;
};
hipError_t launch_select(const rorbk_handle_s *h, const SelectArgs &a, hipStream_t s);

// rhs: rI (forward) or -(sum of partials) (adjoint)
hipError_t launch_chol_solve(const rorbk_handle_s *h, const double *Gpart, int K,
                             const double *rI, const double *Pin, double *y,
                             hipStream_t s);

hipError_t launch_cast_f64_to_f32(const double *src, float *dst, int64_t n,
                                  hipStream_t s);
hipError_t launch_axpy_f32_to_f64(const float *d, double *x, int64_t n,
                                  hipStream_t s);
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s);
hipError_t launch_set_refine_ctrl(Ctrl *c, double tol, double eta,
                                  const double *rout2, double outer_bnorm2,
                                  hipStream_t s);
hipError_t launch_init_ctrl(Ctrl *c, double tol, const double *bnorm2, hipStream_t s);
hipError_t launch_set_thr(Ctrl *c, double thr, hipStream_t s);
hipError_t launch_axpy_f64(const double *d, double *x, int64_t n, hipStream_t s);
// flexible AB-GMRES (Algorithm 3): start vector, one outer step (MGS + Givens),
// final update x += Z y
hipError_t launch_gmres_start(const double *b, const double *axp, int nseg, int64_t m,
                              double *v1, double *g, double *out, hipStream_t s);
hipError_t launch_gmres_step(double *V, int64_t m, int k, const double *axp, int nseg,
                             double *hcol, int M1, double *R, double *cs, double *sn, double *g,
                             double *est, double *part /* 256 doubles */, hipStream_t s);
hipError_t launch_gmres_update(const double *Z, int64_t n, const double *R, const double *g,
                               int kend, int M1, double *x, hipStream_t s);
// initial solution (Algorithm 2): y = column sums of the k x n centroids
hipError_t launch_colsum(const double *cen, int64_t k, int64_t n, double *y, hipStream_t s);
// coefficient from b and the products A y (axp), then x = coefficient * y
hipError_t launch_alg2(const void *b, int vec, const double *axp, int nseg, int64_t m,
                       const double *y, double *coef, void *x, int64_t n, hipStream_t s);

// large-block path (dense): block step, greedy solve, stored inverses
hipError_t launch_step_big(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s);
hipError_t launch_big_chol_solve(const rorbk_handle_s *h, const double *Gpart, int K,
                                 const double *rI, const double *Pin, double *y, hipStream_t s);
hipError_t launch_big_block_inverses(const rorbk_handle_s *h, const double *Gs, int64_t kp,
                                     int32_t *d_fail, hipStream_t s);
hipError_t launch_gram_big(const rorbk_handle_s *h, const void *A, int dt, const int32_t *idx,
                           int K, double *Gpart, hipStream_t s);
// column form: stored inverses (A_t^T A_t + lambda I)^{-1} and the greedy solve
// dx = (A_I^T A_I + lambda I)^{-1} A_I^T r_I (also copies x for the apply kernel)
hipError_t launch_col_block_inverses(const rorbk_handle_s *h, const void *A, int dt,
                                     int32_t *d_fail, hipStream_t s);
// column form, adjoint of one step: y = -A_S (A_S^T A_S + lambda I)^{-1} g' and
// gb[S] -= y (the caller then applies x += A_S^T y with ymode 3)
hipError_t launch_col_adjoint(const rorbk_handle_s *h, const RowSel &rs, int vec, const void *gx,
                              void *gb, double *yout, hipStream_t s);
hipError_t launch_col_greedy(const rorbk_handle_s *h, const void *A, int dt, int aligned, int vec,
                             void *x, const int32_t *I, int K, const double *rI, double *dx,
                             hipStream_t s);

// format-specific block step, residual products and greedy Gram
hipError_t launch_step_dense(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s);
hipError_t launch_residual_dense(const rorbk_handle_s *h, const void *A, int dt,
                                 int aligned, int vec, const void *x, double *axp,
                                 hipStream_t s);
hipError_t launch_residual_dense_side(const rorbk_handle_s *h, const void *A, int dt,
                                      int aligned, int vec, const void *x, double *axp,
                                      const XgSide &side, hipStream_t s);
// fused forward steps (dense, blocks of at most RORBK_FWD_MAX_BLOCK rows)
struct FwdArgs {
    const void *A;        // matrix values (dtype dt)
    int dt;
    int aligned;
    int vec;
    const void *b;        // right-hand side (vector type)
    void *x;              // iterate (vector type)
    const int32_t *I;     // greedy rows (greedy: NULL for products only; samp3: the
                          // chain form's greedy rows, NULL for none)
    const double *y;      // greedy solution y_I
    int64_t tau_index;    // first draw of the iteration (samp3) or of the next one (greedy; < 0: none)
    const double *xg;     // cross-Grams of the iteration (samp3)
};
hipError_t launch_fwd_greedy(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s);
hipError_t launch_fwd_samp3(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s);
hipError_t launch_xgram(const rorbk_handle_s *h, const void *A, int dt, int aligned, int64_t ti,
                        double *out, int waves, hipStream_t s);
int fwd_xgram_jobs(int bmax);
// chain form: the Grams after the selection (greedy Gram and C = A_S' A_I^T in
// column chunks)
hipError_t launch_gram_chain(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                             const int32_t *I, int64_t ti, double *G, hipStream_t s);
// ckst (may be NULL): a checkpoint's chain state, I (raw int32) in doubles
// [0, 32), y in [32, 96), the next z in [96, 96 + 3 * RORBK_FWD_MAX_BLOCK)
constexpr int CKST_DOUBLES = 320;
static_assert(96 + 3 * RORBK_FWD_MAX_BLOCK <= CKST_DOUBLES, "a checkpoint's chain state fits");
// the greedy solve, the next z, the next sampled steps and the combined update
// in one launch (a.I: greedy rows, a.tau_index / a.xg: iteration it + 1)
hipError_t launch_fwd_chain(const rorbk_handle_s *h, const FwdArgs &a, const void *r,
                            double *ckst, hipStream_t s);
hipError_t launch_gram_dense(const rorbk_handle_s *h, const void *A, int dt,
                             const int32_t *idx, int K, double *Gpart, hipStream_t s);
hipError_t launch_step_csr(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s);
hipError_t launch_residual_csr(const rorbk_handle_s *h, const void *vals, int dt, int vec,
                               const void *x, double *axp, hipStream_t s);
hipError_t launch_gram_csr(const rorbk_handle_s *h, const void *vals, int dt,
                           const int32_t *idx, int K, double *Gpart, hipStream_t s);

}  // namespace rorbk
