// k_dense.hip -- ROR-BK kernels for a dense row-major matrix (FP64, FP32 or
// BF16 storage): the fused block step, the greedy block's Gram, and the setup
// (centroid cosines, proposal, block inverses).  The residual pass is in
// k_resid.hip.
#include "rorbk_device.h"
#include "gram_tiles.h"

namespace rorbk {

// ------------------------------------------------------------ block step --
// One regularised block update (Lemma 2's update rule, Algorithm 1) fused with
// the partial products of the next step.  Workgroup w owns the columns
// [w*wu, (w+1)*wu), split into 128-column slabs; a slab is read by NV lanes
// (16 bytes each) per row, and 16 row groups share the rows of a step:
//   1. (ymode 0) r_S = b_S - sum_ch Pin[ch][.] (chunk order), y = H_t r_S with
//      the stored inverse H_t of block t; (ymode 1) y given;
//   2. x[cols] += A_S[:, cols]^T y (row groups summed in group order);
//   3. Pout[w][p] = A_{S'}[p, cols] . x[cols] for the next step's rows S'.
// Every independent load (both row sets' first slab, the partials, the stored
// inverse) is issued before the first barrier, so a step costs a few memory
// round trips.  With b == NULL the step is the adjoint one (see the backward
// pass): then workgroup 0 also accumulates gb[S] -= y.
struct StepP {
    const void *A;
    int64_t ld, m, n, q, rem;
    const int32_t *tau;
    RowSel cur;
    int ymode;
    const double *Pin;
    int nch;
    int bmax;
    const double *H;
    const void *b;
    void *x;
    void *gb;
    const double *ygiven;
    RowSel nxt;
    double *Pout;
    int64_t wu;
    const Ctrl *ctrl;
};

constexpr int STEP_T = 512;  // threads of the block step

// Workgroup barrier that orders LDS only: global loads issued before it stay
// in flight across it (used where the barrier protects LDS data alone).
__device__ __forceinline__ void lds_barrier() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "workgroup", "local");
    __builtin_amdgcn_s_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "workgroup", "local");
}

// row groups of the block step for storage T (8 for FP64, 16 FP32, 32 BF16)
template <typename T>
constexpr int step_groups() { return STEP_T / (128 / Tr<T>::VW); }

template <typename T, typename V, bool AL, int RPT, bool MS>
__global__ __launch_bounds__(STEP_T) void k_step_dense(StepP p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int NV = 128 / VW;       // lanes across a slab
    constexpr int G = step_groups<T>();
    constexpr int NT = STEP_T;
    constexpr int TPR = NT / 128;      // threads per row in the y phase
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const V *__restrict__ b = (const V *)p.b;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;

    int tc = -1, cnt = 0, ncnt = 0;
    int64_t cst = 0, nst = 0;
    if (p.cur.kind == 0) {
        tc = p.tau[p.cur.tau_index];
        cst = blk_start(tc, p.q, p.rem);
        cnt = blk_rows(tc, p.q, p.rem);
    } else if (p.cur.kind == 1) {
        cnt = p.cur.count;
    }
    if (p.nxt.kind == 0) {
        const int tn = p.tau[p.nxt.tau_index];
        nst = blk_start(tn, p.q, p.rem);
        ncnt = blk_rows(tn, p.q, p.rem);
    } else if (p.nxt.kind == 1) {
        ncnt = p.nxt.count;
    }
    if (p.ctrl->done) return;
    const bool upd = p.ymode != 2;
    const int64_t c0 = (int64_t)blockIdx.x * p.wu;
    const int64_t c1 = (c0 + p.wu < p.n) ? c0 + p.wu : p.n;
    const int wcols = (int)(c1 - c0);

    __shared__ V s_x[1024];
    __shared__ V s_red[G][128];
    __shared__ double s_r[MAXB], s_y[MAXB];

    int32_t crow[RPT], nrow[RPT];   // row ids (m < 2^31), -1 = none
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int qq = g + G * r;
        crow[r] = (upd && qq < cnt) ? (p.cur.kind == 1 ? p.cur.idx[qq] : (int32_t)(cst + qq)) : -1;
        nrow[r] = (qq < ncnt) ? (p.nxt.kind == 1 ? p.nxt.idx[qq] : (int32_t)(nst + qq)) : -1;
    }
    uvec4 ua[RPT], un[RPT];
    const uvec4 zero4 = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int64_t col = c0 + (int64_t)v * VW;
        ua[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, col, c1,
                                    crow[r] >= 0, A, c0);
        un[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, col, c1,
                                    nrow[r] >= 0, A, c0);
    }
    for (int c = tid; c < wcols; c += NT) s_x[c] = x[c0 + c];

    if (p.ymode == 0) {
        const double *__restrict__ H = p.H + blk_hoff(tc, p.q, p.rem);
        // prefetch the first HP stored-inverse terms of row tid / TPR
        constexpr int HP = (64 / TPR < 16) ? 64 / TPR : 16;
        double hpre[HP];
        {
            const int i = tid / TPR, qd = tid % TPR;
#pragma unroll
            for (int u = 0; u < HP; ++u) {
                const int j = qd + TPR * u;
                hpre[u] = (i < cnt && j < cnt) ? H[(int64_t)j * cnt + i] : 0.0;
            }
        }
        for (int base = 0; base < cnt; base += 128) {
            const int i = base + tid / TPR, qd = tid % TPR;
            double s = 0.0, bi = 0.0;
            if (i < cnt) {
                const int64_t row = (p.cur.kind == 1) ? (int64_t)p.cur.idx[i] : cst + i;
                bi = b ? (double)b[row] : 0.0;
                for (int cb = 0; cb < p.nch; cb += 8 * TPR) {
                    double t[8];
#pragma unroll
                    for (int u = 0; u < 8; ++u) {
                        const int ch = cb + qd + TPR * u;
                        t[u] = (ch < p.nch) ? p.Pin[(int64_t)ch * p.bmax + i] : 0.0;
                    }
#pragma unroll
                    for (int u = 0; u < 8; ++u) s += t[u];
                }
            }
            s = group_sum(s, TPR);
            if (i < cnt && qd == 0) s_r[i] = bi - s;
        }
        __syncthreads();
        for (int base = 0; base < cnt; base += 128) {
            const int i = base + tid / TPR, qd = tid % TPR;
            double s = 0.0;
            if (i < cnt) {
                for (int jb = 0; jb < cnt; jb += HP * TPR) {
                    double t[HP];
#pragma unroll
                    for (int u = 0; u < HP; ++u) {
                        const int j = jb + qd + TPR * u;
                        t[u] = (base == 0 && jb == 0) ? hpre[u]
                               : ((j < cnt) ? H[(int64_t)j * cnt + i] : 0.0);
                    }
#pragma unroll
                    for (int u = 0; u < HP; ++u) {
                        const int j = jb + qd + TPR * u;
                        if (j < cnt) s = __builtin_fma(t[u], s_r[j], s);
                    }
                }
            }
            s = group_sum(s, TPR);
            if (i < cnt && qd == 0) s_y[i] = s;
        }
        __syncthreads();
    } else {
        if (p.ymode == 1)
            for (int i = tid; i < cnt; i += NT) s_y[i] = p.ygiven[i];
        __syncthreads();
    }
    if (p.gb && upd && blockIdx.x == 0) {
        V *gb = (V *)p.gb;
        for (int i = tid; i < cnt; i += NT) {
            const int64_t row = (p.cur.kind == 1) ? (int64_t)p.cur.idx[i] : cst + i;
            gb[row] -= (V)s_y[i];
        }
    }

    V yv[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) {
        const int qq = g + G * r;
        yv[r] = (upd && qq < cnt) ? (V)s_y[qq] : (V)0;
    }
    V pacc[RPT];
#pragma unroll
    for (int r = 0; r < RPT; ++r) pacc[r] = (V)0;
    // 128-column sub-slabs in turn.  With several sub-slabs per workgroup
    // (MS) and up to 9 rows per thread the next sub-slab's rows are loaded
    // while this one is reduced (its barriers order LDS only, so the loads
    // stay in flight); otherwise each sub-slab loads its own rows
    constexpr bool PF = MS && RPT <= 9;
    constexpr int RP = PF ? RPT : 1;
    for (int64_t sub = c0; sub < c1; sub += 128) {
        const int64_t col = sub + (int64_t)v * VW;
        const bool more = sub + 128 < c1;   // uniform
        uvec4 ua2[RP], un2[RP];
        if constexpr (PF) {
            if (more) {
                const int64_t coln = col + 128;
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    ua2[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, coln,
                                                 c1, crow[r] >= 0, A, c0);
                    un2[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, coln,
                                                 c1, nrow[r] >= 0, A, c0);
                }
            }
        } else if (sub != c0) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                ua[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, col, c1,
                                            crow[r] >= 0, A, c0);
                un[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, col, c1,
                                            nrow[r] >= 0, A, c0);
            }
        }
        if (upd) {
            V acc[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = (V)0;
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                V a[VW];
                cvt_raw<T, V>(ua[r], a);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] = fmaT(a[e], yv[r], acc[e]);
            }
#pragma unroll
            for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
            if (PF) lds_barrier();
            else __syncthreads();
            if (tid < 128) {
                const int64_t cc = sub + tid;
                if (cc < c1) {
                    V s = (V)0;
                    for (int gg = 0; gg < G; ++gg) s += s_red[gg][tid];
                    s_x[cc - c0] += s;
                }
            }
            if (PF) lds_barrier();
            else __syncthreads();
        }
        if (col < c1) {
#pragma unroll
            for (int r = 0; r < RPT; ++r) {
                V a[VW];
                cvt_raw<T, V>(un[r], a);
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    if (col + e < c1) pacc[r] = fmaT(a[e], s_x[col + e - c0], pacc[r]);
            }
        }
        if constexpr (PF) {
            if (more) {
#pragma unroll
                for (int r = 0; r < RPT; ++r) {
                    ua[r] = ua2[r];
                    un[r] = un2[r];
                }
            }
        }
    }
    if (upd)
        for (int c = tid; c < wcols; c += NT) x[c0 + c] = s_x[c];
    // partial products of the next rows: lane sums staged in LDS, then each
    // row's NV sums added in lane order by one thread
    if (ncnt > 0) {
        __shared__ V s_p[RPT * G * NV];
#pragma unroll
        for (int r = 0; r < RPT; ++r) s_p[(r * G + g) * NV + v] = pacc[r];
        __syncthreads();
        for (int row = tid; row < ncnt; row += NT) {
            const V *pp = s_p + row * NV;   // row = g + G * r  ->  (r * G + g) = row
            V s = (V)0;
            for (int l = 0; l < NV; ++l) s += pp[l];
            p.Pout[(int64_t)blockIdx.x * p.bmax + row] = (double)s;
        }
    }
}

// ------------------------------------------------------------ block Gram --
// Lower triangle of A_S A_S^T (the greedy block's Gram, Algorithm 1) on FP64
// MFMA: grid x = 16 x 16 tiles of the lower triangle, grid y = column chunks;
// the four waves of a workgroup take contiguous quarters of the chunk and are
// summed in wave order.  Output: packed lower partials Gpart[chunk][pk(i,j)].
template <typename T, bool AL>
__global__ __launch_bounds__(256) void k_gram_mfma(const T *__restrict__ A, int64_t ld, int64_t n,
                                                   const int32_t *__restrict__ idx, int K,
                                                   int64_t wg, double *__restrict__ Gpart,
                                                   const Ctrl *__restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    constexpr int E = (sizeof(T) == 8) ? 4 : Tr<T>::VW;
    const int nt = (K + 15) / 16;
    int bi, bj;
    tile_of(blockIdx.x, nt, &bi, &bj);
    const int64_t c0 = (int64_t)blockIdx.y * wg;
    const int64_t c1 = (c0 + wg < n) ? c0 + wg : n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
    const int64_t stepc = 4 * E;
    const int64_t span = ((c1 - c0 + 4 * stepc - 1) / (4 * stepc)) * stepc;
    const int64_t wa = c0 + w * span;
    const int64_t wb = (wa + span < c1) ? wa + span : c1;
    const int64_t ra = (bi * 16 + li < K) ? (int64_t)idx[bi * 16 + li] : -1;
    const int64_t rb = (bj * 16 + li < K) ? (int64_t)idx[bj * 16 + li] : -1;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    if (wa < wb) mfma_gram_tile<T, AL>(A, ld, ra, rb, wa, wb, acc);
    __shared__ double red[4][64][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][lane][r] = acc[r];
    __syncthreads();
    if (w == 0) {
        const int KP = K * (K + 1) / 2;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double s = ((red[0][lane][r] + red[1][lane][r]) + red[2][lane][r]) + red[3][lane][r];
            const int ii = bi * 16 + (lane >> 4) + 4 * r, jj = bj * 16 + li;
            if (ii < K && jj <= ii) Gpart[(int64_t)blockIdx.y * KP + pk(ii, jj)] = s;
        }
    }
}

// ------------------------------------------------------------ launchers --
template <typename T, typename V, bool AL, bool MS>
static hipError_t step_launch_ms(const StepP &p, int nblk, int rpt, hipStream_t s) {
    if (rpt <= 3)
        hipLaunchKernelGGL((k_step_dense<T, V, AL, 3, MS>), dim3(nblk), dim3(STEP_T), 0, s, p);
    else if (rpt <= 5)
        hipLaunchKernelGGL((k_step_dense<T, V, AL, 5, MS>), dim3(nblk), dim3(STEP_T), 0, s, p);
    else if (rpt <= 9)
        hipLaunchKernelGGL((k_step_dense<T, V, AL, 9, MS>), dim3(nblk), dim3(STEP_T), 0, s, p);
    else
        hipLaunchKernelGGL((k_step_dense<T, V, AL, 21, MS>), dim3(nblk), dim3(STEP_T), 0, s, p);
    return hipGetLastError();
}

template <typename T, typename V, bool AL>
static hipError_t step_launch_rpt(const StepP &p, int nblk, int bmax, hipStream_t s) {
    constexpr int G = step_groups<T>();
    const int rpt = (bmax + G - 1) / G;
    if (p.wu > 128) return step_launch_ms<T, V, AL, true>(p, nblk, rpt, s);
    return step_launch_ms<T, V, AL, false>(p, nblk, rpt, s);
}

template <typename T, typename V>
static hipError_t step_typed(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    StepP p;
    p.A = a.A;
    p.ld = L.ld;
    p.m = L.m;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.tau = h->d_tau;
    p.cur = a.cur;
    p.ymode = a.ymode;
    p.Pin = a.Pin;
    p.nch = L.nch_u;
    p.bmax = (int)L.bmax;
    p.H = h->d_H;
    p.b = a.b;
    p.x = a.x;
    p.gb = a.gb;
    p.ygiven = a.ygiven;
    p.nxt = a.nxt;
    p.Pout = a.Pout;
    p.wu = L.wu;
    p.ctrl = h->d_ctrl;
    if (a.aligned) return step_launch_rpt<T, V, true>(p, L.nch_u, (int)L.bmax, s);
    return step_launch_rpt<T, V, false>(p, L.nch_u, (int)L.bmax, s);
}

hipError_t launch_step_dense(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    if (a.vec == VEC_F64) return step_typed<double, double>(h, a, s);
    if (a.dt == RORBK_F32) return step_typed<float, float>(h, a, s);
    return step_typed<bf16_t, float>(h, a, s);
}

template <typename T>
static hipError_t gram_typed(const rorbk_handle_s *h, const void *A, int aligned,
                             const int32_t *idx, int K, double *Gpart, hipStream_t s) {
    const Layout &L = h->L;
    const int nt = (K + 15) / 16;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)L.nch_g);
    if (aligned)
        hipLaunchKernelGGL((k_gram_mfma<T, true>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_gram_mfma<T, false>), grid, dim3(256), 0, s, (const T *)A, L.ld,
                           L.n, idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_gram_dense(const rorbk_handle_s *h, const void *A, int dt, const int32_t *idx,
                             int K, double *Gpart, hipStream_t s) {
    const int al = h->aligned;
    if (dt == RORBK_F64) return gram_typed<double>(h, A, al, idx, K, Gpart, s);
    if (dt == RORBK_F32) return gram_typed<float>(h, A, al, idx, K, Gpart, s);
    return gram_typed<bf16_t>(h, A, al, idx, K, Gpart, s);
}

// ------------------------------------------------------------------ setup --
// Centroids (Section 2: the sum of a block's rows), FP64: thread per column,
// rows added in order.  Grid: x = blocks, y = column groups.
template <typename T>
__global__ __launch_bounds__(256) void k_centroid_dense(const T *__restrict__ A, int64_t ld,
                                                        int64_t n, int64_t q, int64_t rem,
                                                        double *__restrict__ cen) {
    const int64_t t = blockIdx.x;
    const int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= n) return;
    const int64_t r0 = blk_start(t, q, rem);
    const int bt = blk_rows(t, q, rem);
    double s = 0.0;
    for (int i = 0; i < bt; ++i) s += (double)to_v<double>(A[(r0 + i) * ld + c]);
    cen[t * n + c] = s;
}

__global__ __launch_bounds__(256) void k_rownorm(const double *__restrict__ cen, int64_t n,
                                                 double *__restrict__ nrm) {
    __shared__ double sh[4];
    const double *ct = cen + (int64_t)blockIdx.x * n;
    double s = 0.0;
    for (int64_t c = threadIdx.x; c < n; c += blockDim.x) s = __builtin_fma(ct[c], ct[c], s);
    s = block_sum(s, sh);
    if (threadIdx.x == 0) nrm[blockIdx.x] = sqrt(s);
}

// Cosine row sums (Section 2, C(i,j) = |<c_i,c_j>| / (|c_i||c_j|)) from the
// centroid Gram on FP64 MFMA, in two kernels.  k_cos64_part: grid x = lower
// 64 x 64 tiles of the Gram, grid y = column parts of pw columns; each
// workgroup forms its tile over its part (gram64_accumulate: four waves, each
// loaded value feeding four products) and stores the whole tile,
// Dp[(tile * parts + part) * 4096 + i * 64 + j].
template <bool AL>
__global__ __launch_bounds__(256) void k_cos64_part(const double *__restrict__ cen, int64_t k,
                                                    int64_t n, int64_t pw, int ntc,
                                                    double *__restrict__ Dp) {
    int bi, bj;
    tile_of(blockIdx.x, ntc, &bi, &bj);
    if (bi < 0) return;   // uniform, before any barrier
    const int64_t c0 = (int64_t)blockIdx.y * pw;
    const int64_t c1 = (c0 + pw < n) ? c0 + pw : n;
    const int li = threadIdx.x & 15;
    const double *pa[4], *pb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        const int64_t ia = (int64_t)bi * 64 + s2 * 16 + li, ib = (int64_t)bj * 64 + s2 * 16 + li;
        va[s2] = ia < k;
        vb[s2] = ib < k;
        pa[s2] = cen + (va[s2] ? ia : 0) * n;
        pb[s2] = cen + (vb[s2] ? ib : 0) * n;
    }
    dvec4 acc[4][4];
    gram64_accumulate<double, AL>(pa, pb, va, vb, bi == bj, c0, c1, acc);
    gram64_store_tile(acc, Dp + ((int64_t)blockIdx.x * gridDim.y + blockIdx.y) * 4096);
}

// k_cos64_rows: one workgroup per tile (bi, bj).  Entry (i, j) is the sum of
// the parts in part order (on a diagonal tile taken from the lower half,
// (max, min)), normalised to |d| / (|c_i||c_j|) (a zero centroid has C(t,t) = 1
// and C(t,j) = 0) and kept in LDS; thread t takes entries t, t + 256, ...
// Then thread (row, quarter) sums 16 entries in column order and the four
// quarters combine by a fixed butterfly: the row sums -> Sp[i][bj], and
// (bi != bj) the column sums -> Sp[j][bi]; every Sp entry is written once.
__global__ __launch_bounds__(256) void k_cos64_rows(const double *__restrict__ Dp, int parts,
                                                    int64_t k, const double *__restrict__ nrm,
                                                    int ntc, double *__restrict__ Sp) {
    __shared__ double c[64][65];
    __shared__ double s_n[128];   // |c_i| of the tile's rows, then of its columns
    int bi, bj;
    tile_of(blockIdx.x, ntc, &bi, &bj);
    if (bi < 0) return;
    if (threadIdx.x < 128) {
        const int64_t g = (threadIdx.x < 64) ? (int64_t)bi * 64 + threadIdx.x
                                             : (int64_t)bj * 64 + threadIdx.x - 64;
        s_n[threadIdx.x] = (g < k) ? nrm[g] : 0.0;
    }
    const double *D = Dp + (int64_t)blockIdx.x * parts * 4096;
    // the sixteen entries of this thread summed over the parts in part
    // order, the sixteen loads of a part issued together
    double d[16];
#pragma unroll
    for (int u = 0; u < 16; ++u) d[u] = 0.0;
    for (int p = 0; p < parts; ++p) {
        double t[16];
#pragma unroll
        for (int u = 0; u < 16; ++u) {
            const int e0 = (int)threadIdx.x + 256 * u;
            const int row = e0 >> 6, col = e0 & 63;
            const int e = (bi == bj && col > row) ? col * 64 + row : e0;
            t[u] = D[(int64_t)p * 4096 + e];
        }
#pragma unroll
        for (int u = 0; u < 16; ++u) d[u] += t[u];
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 16; ++u) {
        const int e0 = (int)threadIdx.x + 256 * u;
        const int row = e0 >> 6, col = e0 & 63;
        const int64_t ii = (int64_t)bi * 64 + row, jj = (int64_t)bj * 64 + col;
        double v = 0.0;
        if (ii < k && jj < k) {
            const double ni = s_n[row], nj = s_n[64 + col];
            if (ni == 0.0 || nj == 0.0) v = (ii == jj) ? 1.0 : 0.0;
            else v = fabs(d[u]) / (ni * nj);
        }
        c[row][col] = v;
    }
    __syncthreads();
    const int row = threadIdx.x >> 2, qt = threadIdx.x & 3;
    const int64_t ii = (int64_t)bi * 64 + row;
    double rs = 0.0;
    for (int u = 0; u < 16; ++u) rs += c[row][qt * 16 + u];
    rs += __shfl_xor(rs, 1, 64);
    rs += __shfl_xor(rs, 2, 64);
    if (qt == 0 && ii < k) Sp[ii * ntc + bj] = rs;
    if (bi != bj) {
        // thread (column, quarter): rows qt*16 .. qt*16+15 of that column
        const int col = threadIdx.x >> 2;
        const int64_t jj = (int64_t)bj * 64 + col;
        double cs = 0.0;
        for (int u = 0; u < 16; ++u) cs += c[qt * 16 + u][col];
        cs += __shfl_xor(cs, 1, 64);
        cs += __shfl_xor(cs, 2, 64);
        if (qt == 0 && jj < k) Sp[jj * ntc + bi] = cs;
    }
}

// S_t = sum of the tile partials in tile order, Pbar_t = exp(-2 S_t / n)
// (Section 2, the proposal), and W = running sums of Pbar in block order.
// S_t (the |cos| row sums, from the per-tile partials) and pbar_t: one wave
// per block, lane l summing tiles l, l + 64, ... in order, then a fixed
// butterfly.
__global__ __launch_bounds__(256) void k_proposal_rows(const double *__restrict__ Sp,
                                                       int64_t ntile, int64_t k, int64_t n,
                                                       double *__restrict__ S,
                                                       double *__restrict__ pbar) {
    const int64_t t = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    const int lane = threadIdx.x & 63;
    if (t >= k) return;   // uniform per wave
    double s = 0.0;
    for (int64_t j = lane; j < ntile; j += 64) s += Sp[t * ntile + j];
    s = group_sum(s, 64);
    if (lane == 0) {
        S[t] = s;
        pbar[t] = exp(-2.0 * s / (double)n);
    }
}

// W = the running sum of pbar, in block order (one thread; pbar staged in LDS
// by the workgroup first).
__global__ __launch_bounds__(1024) void k_proposal(const double *__restrict__ pbar, int64_t k,
                                                   double *__restrict__ W) {
    __shared__ double sp[8192];
    for (int64_t c0 = 0; c0 < k; c0 += 8192) {
        const int64_t c1 = (c0 + 8192 < k) ? c0 + 8192 : k;
        for (int64_t t = c0 + threadIdx.x; t < c1; t += blockDim.x) sp[t - c0] = pbar[t];
        __syncthreads();
        if (threadIdx.x == 0) {
            double acc = (c0 > 0) ? W[c0 - 1] : 0.0;
            for (int64_t t = c0; t < c1; ++t) {
                acc += sp[t - c0];
                W[t] = acc;
            }
        }
        __syncthreads();
    }
}

// Column parts of the centroid Gram: the count P (at most 32, parts of at
// least 512 columns so that the per-workgroup reduction and store stay small
// beside the products, at most 4096 partial tiles) that spends the fewest
// workgroup rounds per unit of work, ceil(tiles P / ncu) / P (one workgroup
// per CU at a time); each part a multiple of 64 columns.
void cos_parts(int64_t k, int64_t n, int ncu, int64_t *parts, int64_t *pw) {
    const int64_t ntc = (k + 63) / 64, tiles = ntc * (ntc + 1) / 2;
    int64_t pmax = 32;
    if (pmax > n / 512) pmax = n / 512;
    if (pmax > 4096 / tiles) pmax = 4096 / tiles;
    if (pmax < 1) pmax = 1;
    int64_t best = 1;
    for (int64_t p = 2; p <= pmax; ++p) {
        // rounds(p) / p < rounds(best) / best, in integers
        const int64_t rp = (tiles * p + ncu - 1) / ncu, rb = (tiles * best + ncu - 1) / ncu;
        if (rp * best < rb * p) best = p;
    }
    int64_t w = ((n + best - 1) / best + 63) / 64 * 64;
    if (w < 64) w = 64;
    *pw = w;
    *parts = (n + w - 1) / w;
}

int64_t setup_proposal_scratch(int64_t k, int64_t n, int ncu) {
    int64_t parts, pw;
    cos_parts(k, n, ncu, &parts, &pw);
    const int64_t ntc = (k + 63) / 64, tiles = ntc * (ntc + 1) / 2;
    return k * n + k + k * ntc + tiles * parts * 4096;
}

// scratch: cen (k x n), nrm (k), Sp (k x ntc), then the Gram parts
hipError_t launch_proposal_from_centroids(const rorbk_handle_s *h, double *cen, double *nrm,
                                          double *Sp, hipStream_t s) {
    const Layout &L = h->L;
    hipLaunchKernelGGL(k_rownorm, dim3((unsigned)L.k), dim3(256), 0, s, cen, L.n, nrm);
    const int64_t ntc = (L.k + 63) / 64;
    const int64_t tiles = ntc * (ntc + 1) / 2;
    int64_t parts, pw;
    cos_parts(L.k, L.n, h->ncu, &parts, &pw);
    double *Dp = Sp + L.k * ntc;
    const bool al = (L.n % 2) == 0;   // 16-byte rows of the FP64 centroid matrix
    const dim3 grid((unsigned)tiles, (unsigned)parts);
    if (al)
        hipLaunchKernelGGL(k_cos64_part<true>, grid, dim3(256), 0, s, cen, L.k, L.n, pw, (int)ntc,
                           Dp);
    else
        hipLaunchKernelGGL(k_cos64_part<false>, grid, dim3(256), 0, s, cen, L.k, L.n, pw,
                           (int)ntc, Dp);
    hipLaunchKernelGGL(k_cos64_rows, dim3((unsigned)tiles), dim3(256), 0, s, Dp, (int)parts, L.k,
                       nrm, (int)ntc, Sp);
    hipLaunchKernelGGL(k_proposal_rows, dim3((unsigned)((L.k + 3) / 4)), dim3(256), 0, s, Sp, ntc,
                       L.k, L.n, h->d_S, h->d_pbar);
    hipLaunchKernelGGL(k_proposal, dim3(1), dim3(1024), 0, s, h->d_pbar, L.k, h->d_W);
    return hipGetLastError();
}

hipError_t launch_setup_proposal_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                       double *scratch, hipStream_t s) {
    (void)aligned;
    const Layout &L = h->L;
    double *cen = scratch;                      // k * n
    double *nrm = cen + L.k * L.n;              // k
    double *Sp = nrm + L.k;                     // k * ntc
    dim3 grid((unsigned)L.k, (unsigned)((L.n + 255) / 256));
    if (dt == RORBK_F64)
        hipLaunchKernelGGL(k_centroid_dense<double>, grid, dim3(256), 0, s, (const double *)A,
                           L.ld, L.n, L.q, L.rem, cen);
    else if (dt == RORBK_F32)
        hipLaunchKernelGGL(k_centroid_dense<float>, grid, dim3(256), 0, s, (const float *)A, L.ld,
                           L.n, L.q, L.rem, cen);
    else
        hipLaunchKernelGGL(k_centroid_dense<bf16_t>, grid, dim3(256), 0, s, (const bf16_t *)A,
                           L.ld, L.n, L.q, L.rem, cen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_colsum(cen, L.k, L.n, h->d_ysum, s);     // the row sum of A (Algorithm 2)
    if (e != hipSuccess) return e;
    return launch_proposal_from_centroids(h, cen, nrm, Sp, s);
}

// Fixed-block Grams G_t = A_t A_t^T on FP64 MFMA (Section 3.1 stores each
// block's regularised inverse once): grid x = lower 16 x 16 tiles of the
// largest block, grid y = blocks; packed lower output Gs[t][pk(i,j)].
template <typename T, bool AL>
__global__ __launch_bounds__(256) void k_block_gram_mfma(const T *__restrict__ A, int64_t ld,
                                                         int64_t n, int64_t q, int64_t rem,
                                                         int64_t kpmax, double *__restrict__ Gs) {
    const int64_t t = blockIdx.y;
    const int bt = blk_rows(t, q, rem);
    const int64_t r0 = blk_start(t, q, rem);
    const int nt = (bt + 15) / 16;
    int bi, bj;
    tile_of(blockIdx.x, (int)((q + 1 + 15) / 16), &bi, &bj);
    if (bi < 0 || bi >= nt || bj >= nt) return;
    constexpr int E = (sizeof(T) == 8) ? 4 : Tr<T>::VW;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
    const int64_t stepc = 4 * E;
    const int64_t span = ((n + 4 * stepc - 1) / (4 * stepc)) * stepc;
    const int64_t wa = w * span;
    const int64_t wb = (wa + span < n) ? wa + span : n;
    const int64_t ra = (bi * 16 + li < bt) ? r0 + bi * 16 + li : -1;
    const int64_t rb = (bj * 16 + li < bt) ? r0 + bj * 16 + li : -1;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    if (wa < wb) mfma_gram_tile<T, AL>(A, ld, ra, rb, wa, wb, acc);
    __shared__ double red[4][64][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][lane][r] = acc[r];
    __syncthreads();
    if (w == 0) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const double s = ((red[0][lane][r] + red[1][lane][r]) + red[2][lane][r]) + red[3][lane][r];
            const int ii = bi * 16 + (lane >> 4) + 4 * r, jj = bj * 16 + li;
            if (ii < bt && jj <= ii) Gs[t * kpmax + pk(ii, jj)] = s;
        }
    }
}

// The same block Grams on 64 x 64 tiles (gram_tiles.h) for blocks of at least
// 48 rows: grid x = lower 64 x 64 tiles of the largest block, grid
// y = blocks; each workgroup sums its tile over all n columns, with the
// values of the 16 x 16 tile kernel.
template <typename T, bool AL>
__global__ __launch_bounds__(256) void k_block_gram64(const T *__restrict__ A, int64_t ld,
                                                      int64_t n, int64_t q, int64_t rem,
                                                      int64_t kpmax, double *__restrict__ Gs) {
    const int64_t t = blockIdx.y;
    const int bt = blk_rows(t, q, rem);
    const int64_t r0 = blk_start(t, q, rem);
    const int nt = (bt + 63) / 64;
    int bi, bj;
    tile_of(blockIdx.x, (int)((q + 1 + 63) / 64), &bi, &bj);
    if (bi < 0 || bi >= nt || bj >= nt) return;   // uniform, before any barrier
    const int li = threadIdx.x & 15;
    const T *pa[4], *pb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        const int ia = bi * 64 + s2 * 16 + li, ib = bj * 64 + s2 * 16 + li;
        va[s2] = ia < bt;
        vb[s2] = ib < bt;
        pa[s2] = A + (r0 + (va[s2] ? ia : 0)) * ld;
        pb[s2] = A + (r0 + (vb[s2] ? ib : 0)) * ld;
    }
    dvec4 acc[4][4];
    gram64_accumulate<T, AL, true>(pa, pb, va, vb, bi == bj, 0, n, acc);
    gram64_store(acc, bi, bj, bt, Gs + t * kpmax);
}

// Stored inverse of each fixed block: (G_t + lambda I)^{-1} from the LDL^T
// factor (LDS), column j by thread j (forward with unit L, scale by D^{-1},
// backward with L^T), written row-major (the inverse is symmetric).
template <int MT>
__global__ __launch_bounds__(256) void k_block_inverse(const double *__restrict__ Gs, int64_t kpmax,
                                                       int64_t q, int64_t rem, double lambda,
                                                       double *__restrict__ H,
                                                       int32_t *__restrict__ fail) {
    __shared__ double Gp[PACKED_MAX];
    __shared__ double z[MAXB];
    __shared__ double colbuf[2 * MAXB];
    __shared__ double invd[MAXB];
    const int64_t t = blockIdx.x;
    const int K = blk_rows(t, q, rem);
    const int KP = K * (K + 1) / 2;
    for (int f = threadIdx.x; f < KP; f += blockDim.x) Gp[f] = Gs[t * kpmax + f];
    for (int i = threadIdx.x; i < K; i += blockDim.x) z[i] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += blockDim.x) Gp[pk(i, i)] += lambda;
    __syncthreads();
    if (!ldl_solve<MT>(Gp, z, K, colbuf)) {
        if (threadIdx.x == 0) *fail = 1;
        return;
    }
    for (int i = threadIdx.x; i < K; i += blockDim.x) invd[i] = 1.0 / Gp[pk(i, i)];
    __syncthreads();
    double *Hb = H + blk_hoff(t, q, rem);
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        double *h = Hb + (int64_t)j * K;
        for (int i = 0; i < j; ++i) h[i] = 0.0;
        for (int i = j; i < K; ++i) {          // unit lower: z_i = e_j - sum l_ip z_p
            double s = (i == j) ? 1.0 : 0.0;
            for (int p2 = j; p2 < i; ++p2) s -= Gp[pk(i, p2)] * invd[p2] * h[p2];
            h[i] = s;
        }
        for (int i = j; i < K; ++i) h[i] *= invd[i];
        for (int i = K - 1; i >= 0; --i) {     // L^T h = D^{-1} z
            double s = h[i];
            for (int p2 = i + 1; p2 < K; ++p2) s -= Gp[pk(p2, i)] * invd[i] * h[p2];
            h[i] = s;
        }
    }
}

// Blocks of at most KM rows: the same LDL^T (ldl_solve on 4 x 4 tiles), then the inverse in
// LDS: M = L^{-1} column by column (four threads per column j:
// m_ij = [i == j] - sum_{p<i} l_ip m_pj, thread q of the four summing the
// p = q mod 4 terms in order, the four partials added by a fixed butterfly;
// all columns run the same i, so l_ip is a broadcast read), and
// H = M^T D^{-1} M entry by entry (h_ij = sum_{p >= max(i,j)} (m_pi m_pj) / d_p,
// the product taken in an order-free way so that H is exactly symmetric),
// written row-major with consecutive threads on consecutive entries.
template <int KM>
__global__ __launch_bounds__(4 * KM) void k_block_inverse_lds(const double *__restrict__ Gs,
                                                           int64_t kpmax, int64_t q, int64_t rem,
                                                           double lambda, double *__restrict__ H,
                                                           int32_t *__restrict__ fail) {
    __shared__ double Gp[KM * (KM + 1) / 2];
    __shared__ double z[KM];
    __shared__ double colbuf[2 * MAXB];
    __shared__ double invd[KM];
    __shared__ double M[KM][KM + 1];
    const int64_t t = blockIdx.x;
    const int K = blk_rows(t, q, rem);
    const int KP = K * (K + 1) / 2;
    for (int f = threadIdx.x; f < KP; f += blockDim.x) Gp[f] = Gs[t * kpmax + f];
    for (int i = threadIdx.x; i < K; i += blockDim.x) z[i] = 0.0;
    __syncthreads();
    for (int i = threadIdx.x; i < K; i += blockDim.x) Gp[pk(i, i)] += lambda;
    __syncthreads();
    static_assert(((KM + 3) / 4) * ((KM + 3) / 4 + 1) / 2 <= 256, "4 x 4 tiles cover the block");
    if (!ldl_solve<4>(Gp, z, K, colbuf)) {
        if (threadIdx.x == 0) *fail = 1;
        return;
    }
    for (int i = threadIdx.x; i < K; i += blockDim.x) invd[i] = 1.0 / Gp[pk(i, i)];
    __syncthreads();
    // unit lower factor: l_ip = g_ip / d_p (i > p)
    for (int f = threadIdx.x; f < KP; f += blockDim.x) {
        int i = 0;
        while (pk(i + 1, 0) <= f) ++i;
        const int p2 = f - pk(i, 0);
        if (p2 < i) Gp[f] *= invd[p2];
    }
    __syncthreads();
    // M = L^{-1}, four threads per column (consecutive lanes of one wave)
    {
        const int j = threadIdx.x >> 2, qq = threadIdx.x & 3;
        const int jc = (j < K) ? j : 0;
        for (int i = 0; i < K; ++i) {
            double part = 0.0;
            for (int p2 = qq; p2 < i; p2 += 4) part = __builtin_fma(Gp[pk(i, p2)], M[p2][jc], part);
            part += __shfl_xor(part, 1, 4);
            part += __shfl_xor(part, 2, 4);
            const double mij = (i > j) ? -part : ((i == j) ? 1.0 : 0.0);
            if (j < K && qq == (i & 3)) M[i][j] = mij;
        }
    }
    __syncthreads();
    // H = M^T D^{-1} M
    double *Hb = H + blk_hoff(t, q, rem);
    for (int e = threadIdx.x; e < K * K; e += blockDim.x) {
        const int i = e / K, j = e - i * K;
        const int p0 = i > j ? i : j;
        double sacc = 0.0;
        for (int p2 = p0; p2 < K; ++p2) sacc = __builtin_fma(M[p2][i] * M[p2][j], invd[p2], sacc);
        Hb[e] = sacc;
    }
}

hipError_t launch_block_inverses_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                       int32_t *d_fail, hipStream_t s) {
    const Layout &L = h->L;
    const int64_t kp = L.bmax * (L.bmax + 1) / 2;
    double *Gs = nullptr;
    hipError_t e = hipMallocAsync((void **)&Gs, sizeof(double) * (size_t)(kp * L.k), s);
    if (e != hipSuccess) return e;
    // 64 x 64 tiles once a block fills most of one (48 rows: the 16 x 16 form
    // has as many products then, each a dependent MFMA chain of its own)
    const bool t64 = L.bmax >= 48;
    const int nt = (int)(t64 ? (L.bmax + 63) / 64 : (L.bmax + 15) / 16);
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)L.k);
#define RORBK_BG(T)                                                                             \
    do {                                                                                        \
        if (t64 && aligned)                                                                     \
            hipLaunchKernelGGL((k_block_gram64<T, true>), grid, dim3(256), 0, s,                \
                               (const T *)A, L.ld, L.n, L.q, L.rem, kp, Gs);                    \
        else if (t64)                                                                           \
            hipLaunchKernelGGL((k_block_gram64<T, false>), grid, dim3(256), 0, s,               \
                               (const T *)A, L.ld, L.n, L.q, L.rem, kp, Gs);                    \
        else if (aligned)                                                                       \
            hipLaunchKernelGGL((k_block_gram_mfma<T, true>), grid, dim3(256), 0, s,             \
                               (const T *)A, L.ld, L.n, L.q, L.rem, kp, Gs);                    \
        else                                                                                    \
            hipLaunchKernelGGL((k_block_gram_mfma<T, false>), grid, dim3(256), 0, s,            \
                               (const T *)A, L.ld, L.n, L.q, L.rem, kp, Gs);                    \
    } while (0)
    if (dt == RORBK_F64) RORBK_BG(double);
    else if (dt == RORBK_F32) RORBK_BG(float);
    else RORBK_BG(bf16_t);
#undef RORBK_BG
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_block_inverses_from_grams(h, Gs, kp, d_fail, s);
    hipError_t e2 = hipFreeAsync(Gs, s);
    return e != hipSuccess ? e : e2;
}

hipError_t launch_block_inverses_from_grams(const rorbk_handle_s *h, const double *Gs, int64_t kp,
                                            int32_t *d_fail, hipStream_t s) {
    const Layout &L = h->L;
    if (L.bmax > MAXB) return launch_big_block_inverses(h, Gs, kp, d_fail, s);
    if (L.bmax <= 64)
        hipLaunchKernelGGL(k_block_inverse_lds<64>, dim3((unsigned)L.k), dim3(256), 0, s, Gs, kp,
                           L.q, L.rem, h->lambda, h->d_H, d_fail);
    else if (L.bmax <= 72)
        hipLaunchKernelGGL(k_block_inverse_lds<72>, dim3((unsigned)L.k), dim3(288), 0, s, Gs, kp,
                           L.q, L.rem, h->lambda, h->d_H, d_fail);
    else
        hipLaunchKernelGGL(k_block_inverse<8>, dim3((unsigned)L.k), dim3(256), 0, s, Gs, kp, L.q,
                           L.rem, h->lambda, h->d_H, d_fail);
    return hipGetLastError();
}

}  // namespace rorbk
