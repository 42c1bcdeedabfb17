// k_fwd.hip -- the forward iteration's block steps for dense row-major
// matrices whose blocks have at most FWD_B rows (row form): the three sampled
// updates of an outer iteration (Algorithm 1, inner loop) in one launch, the
// greedy update fused with the next iteration's products, the cross-Grams
// of the three sampled blocks, and the chain form in which the greedy update
// of iteration it and the sampled updates of iteration it + 1 share one pass.
//
// The three sampled steps x1 = x0 + A1^T y1, x2 = x1 + A2^T y2,
// x3 = x2 + A3^T y3 with y_l = H_l (b_l - A_l x_{l-1}) (Lemma 2's update
// rule, H_l the stored inverse of block l, Section 3.1) need A_2 x1 and
// A_3 x2.  Since A_2 x1 = A_2 x0 + (A_2 A_1^T) y1 and
// A_3 x2 = A_3 x0 + (A_3 A_1^T) y1 + (A_3 A_2^T) y2, the three products
// A_l x0 (one pass, partial sums per column slab) and the cross-Grams
// A_2 A_1^T, A_3 A_1^T, A_3 A_2^T (which do not depend on x and are formed one
// iteration ahead) give y1, y2, y3 in a short chain of small matrix-vector
// products, and x3 = x0 + A_1^T y1 + A_2^T y2 + A_3^T y3 is one more pass.  The
// same iterate results in exact arithmetic; the roundings differ from three
// separate steps.
#include "ldl_blk.h"
#include "rorbk_device.h"
#include "xgram.h"

namespace rorbk {

constexpr int FWD_T = 512;      // threads of the step kernels

// The three blocks drawn at tau[ti .. ti+2]: first row and row count of each
// (named scalars, so that no index into them is computed at run time).
struct Blk3 {
    int64_t s0, s1, s2;
    int c0, c1, c2;
};

__device__ __forceinline__ void blocks3(const int32_t *__restrict__ tau, int64_t ti, int64_t q,
                                        int64_t rem, Blk3 &B) {
    const int64_t t0 = tau[ti], t1 = tau[ti + 1], t2 = tau[ti + 2];
    B.s0 = blk_start(t0, q, rem);
    B.s1 = blk_start(t1, q, rem);
    B.s2 = blk_start(t2, q, rem);
    B.c0 = blk_rows(t0, q, rem);
    B.c1 = blk_rows(t1, q, rem);
    B.c2 = blk_rows(t2, q, rem);
}

// Row qq of the three blocks taken in order: its block l, offset i and row.
__device__ __forceinline__ void split3(const Blk3 &B, int qq, int *l, int *i, int64_t *row) {
    const bool a = qq >= B.c0, b = qq >= B.c0 + B.c1;
    *l = (int)a + (int)b;
    *i = qq - (a ? B.c0 : 0) - (b ? B.c1 : 0);
    // offsets added under two independent selects (a three-way select can be
    // turned into an indexed table in scratch memory)
    *row = B.s0 + (a ? B.s1 - B.s0 : 0) + (b ? B.s2 - B.s1 : 0) + *i;
}

// Columns of one sub-slab: 64 for FP64 storage (16 row groups of 32 lanes
// keep the three-block row set in registers), 128 otherwise.
template <typename T>
__host__ __device__ constexpr int fwd_swc() { return sizeof(T) == 8 ? 64 : 128; }

template <typename T, bool AL, int NW>
__global__ __launch_bounds__(64 * NW) void k_xgram(const T *__restrict__ A, int64_t ld, int64_t n,
                                                   const int32_t *__restrict__ tau, int64_t ti,
                                                   int64_t q, int64_t rem, int bmax,
                                                   double *__restrict__ out,
                                                   const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    xgram_tile<T, AL, NW>(A, ld, n, tau, ti, q, rem, bmax, blockIdx.x, out);
}

// ------------------------------------------------- Grams of the chain form --
// After the selection of iteration it, with the blocks S' drawn for iteration
// it + 1 at tau[ti .. ti+2]: the greedy Gram A_I A_I^T (packed lower) and
// C = A_{S'} A_I^T (C[(l * FWD_B + i) * 64 + j] = <row i of block l, row I_j>),
// as partial sums over nch column chunks (chunk ch at G + ch * K(K+1)/2 and
// C + ch * CHAIN_C).  Since A_{S'} (x + A_I^T y) = A_{S'} x + C y, the next
// iteration's z = b_{S'} - A_{S'} x_new = r_{S'} - C y follows from the
// residual r of this iteration (taken at x, before the greedy step) once y is
// known, with no pass over x in between.  One 16 x 16 tile of one chunk per
// workgroup: the GC_W waves take consecutive column ranges (multiples of the
// MFMA step) and are summed in wave order.  (The cross-Grams of S' do not
// depend on I and are formed by spare workgroups of the selection.)
constexpr int GC_W = 8;
constexpr int CHAIN_C = 3 * FWD_B * 64;   // doubles of one chunk of C

struct GramChainP {
    const void *A;
    int64_t ld, n, q, rem;
    int bmax;
    const int32_t *I;
    int K;
    const int32_t *tau;
    int64_t ti;
    int64_t wc;     // columns per chunk (a multiple of 32)
    double *G;      // [nch][K (K + 1) / 2], packed lower
    double *C;      // [nch][3 * FWD_B][64]
    const Ctrl *ctrl;
};

__host__ __device__ inline int gram_chain_tiles(int K, int bmax) {
    const int nt = (K + 15) / 16, nb = (bmax + 15) / 16;
    return nt * (nt + 1) / 2 + 3 * nb * nt;
}

template <typename T, bool AL>
__global__ __launch_bounds__(64 * GC_W) void k_gram_chain(GramChainP p) {
    // the stop flag is read together with the row indices: one memory
    // latency before the row loads instead of two
    const int stop =
        __hip_atomic_load(&p.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    constexpr int E = (sizeof(T) == 8) ? 4 : Tr<T>::VW;
    const T *__restrict__ A = (const T *)p.A;
    const int K = p.K;
    const int nt = (K + 15) / 16, ntg = nt * (nt + 1) / 2;
    const int nb = (p.bmax + 15) / 16, nc = 3 * nb * nt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
    const int job = (int)blockIdx.x % (ntg + nc), ch = (int)blockIdx.x / (ntg + nc);
    int kind, bi, bj, l = 0, ca = K;
    int64_t ra, rb;
    if (job < ntg) {                 // greedy Gram, lower tiles
        kind = 0;
        tile_of(job, nt, &bi, &bj);
    } else {                         // C: block l of S' against I
        kind = 1;
        const int c = job - ntg;
        l = c / (nb * nt);
        const int rest = c - l * nb * nt;
        bi = rest / nt;
        bj = rest - bi * nt;
    }
    // the greedy rows of this lane, read with clamped indices (no branch
    // around the loads) before the sampled block's start
    const int ia = bi * 16 + li, ib = bj * 16 + li;
    const int32_t Ia = p.I[ia < K ? ia : K - 1];
    const int32_t Ib = p.I[ib < K ? ib : K - 1];
    rb = (ib < K) ? (int64_t)Ib : -1;
    if (kind == 0) {
        ra = (ia < K) ? (int64_t)Ia : -1;
    } else {
        const int64_t t = p.tau[p.ti + l];
        ca = blk_rows(t, p.q, p.rem);
        if (bi * 16 >= ca) return;   // uniform: a tile past the block
        ra = (ia < ca) ? blk_start(t, p.q, p.rem) + ia : -1;
    }
    if (stop) return;
    const int64_t c0 = (int64_t)ch * p.wc;
    const int64_t c1 = (c0 + p.wc < p.n) ? c0 + p.wc : p.n;
    const int64_t stepc = 4 * E;
    const int64_t span = ((c1 - c0 + GC_W * stepc - 1) / (GC_W * stepc)) * stepc;
    const int64_t wa = c0 + (int64_t)w * span;
    const int64_t wb = (wa + span < c1) ? wa + span : c1;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    if (wa < wb) mfma_gram_tile<T, AL>(A, p.ld, ra, rb, wa, wb, acc);
    __shared__ double red[GC_W][64][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][lane][r] = acc[r];
    __syncthreads();
    if (w != 0) return;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
        double s = red[0][lane][r];
#pragma unroll
        for (int v = 1; v < GC_W; ++v) s += red[v][lane][r];
        const int ii = bi * 16 + (lane >> 4) + 4 * r, jj = bj * 16 + li;
        if (kind == 0) {
            if (ii < K && jj <= ii) p.G[(int64_t)ch * (K * (K + 1) / 2) + pk(ii, jj)] = s;
        } else {
            if (ii < ca && jj < K) p.C[(int64_t)ch * CHAIN_C + (l * FWD_B + ii) * 64 + jj] = s;
        }
    }
}

// ------------------------------------------ greedy update + next products --
// x[cols] += A_I[:, cols]^T y_I (the greedy step, y_I given) over column slabs
// of wu columns per workgroup, then the partial products of the next
// iteration's three sampled blocks on the updated slab:
// Pout[w][l * bmax + i] = A_{S_l}[i, cols] . x[cols].  With I == NULL only the
// products are formed (the first iteration of a run); with tau_next < 0 only
// the update (the last iteration).  Rows are spread over G row groups of NV
// lanes (16 bytes each across a sub-slab of fwd_swc columns): the current rows RC per
// thread, the next rows RN per thread.  Every load of both row sets' first
// sub-slab is issued before the first barrier; with PF the next sub-slab's
// rows load while the current one is reduced.  The last workgroup to finish
// (device-scope acquire-release counter) then forms
// z[l * FWD_B + i] = b_{S_l}[i] - sum_ch Pout[ch][l * bmax + i] (chunk order;
// zero in unused slots), the start of the next three-step chain.
struct FwdGreedyP {
    const void *A;
    int64_t ld, n, q, rem;
    int bmax;
    const int32_t *tau;
    int64_t tau_next;
    const int32_t *I;
    int K;
    const double *y;
    void *x;
    double *Pout;
    int64_t wu;
    const Ctrl *ctrl;
    const void *b;         // right-hand side (vector type)
    double *z3;            // z of the next iteration's blocks, slots l * FWD_B + i
    uint32_t *counter;     // workgroups done (0 between launches)
};

template <typename T, typename V, bool AL, int RC, int RN, bool MS>
__global__ __launch_bounds__(FWD_T) void k_fwd_greedy(FwdGreedyP p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int SWC = fwd_swc<T>();
    constexpr int NV = SWC / VW;
    constexpr int G = FWD_T / NV;
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;
    Blk3 B = {0, 0, 0, 0, 0, 0};
    if (p.tau_next >= 0) blocks3(p.tau, p.tau_next, p.q, p.rem, B);
    const int ncnt = B.c0 + B.c1 + B.c2;
    const int cnt = p.I ? p.K : 0;
    if (p.ctrl->done) return;
    const int64_t c0 = (int64_t)blockIdx.x * p.wu;
    const int64_t c1 = (c0 + p.wu < p.n) ? c0 + p.wu : p.n;
    const int wcols = (int)(c1 - c0);

    __shared__ V s_x[1024];
    __shared__ V s_red[G][SWC];
    __shared__ double s_y[FWD_B];

    int32_t crow[RC], nrow[RN];
    int nidx[RN];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int qq = g + G * r;
        crow[r] = (qq < cnt) ? p.I[qq] : -1;
    }
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        const int qq = g + G * r;
        nrow[r] = -1;
        nidx[r] = 0;
        if (qq < ncnt) {
            int l, i;
            int64_t row;
            split3(B, qq, &l, &i, &row);
            nrow[r] = (int32_t)row;
            nidx[r] = l * p.bmax + i;
        }
    }
    const uvec4 zero4 = {0u, 0u, 0u, 0u};
    uvec4 ua[RC], un[RN];
    {
        const int64_t col = c0 + (int64_t)v * VW;
#pragma unroll
        for (int r = 0; r < RC; ++r)
            ua[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, col, c1,
                                        crow[r] >= 0, A, c0);
#pragma unroll
        for (int r = 0; r < RN; ++r)
            un[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, col, c1,
                                        nrow[r] >= 0, A, c0);
    }
    for (int c = tid; c < wcols; c += FWD_T) s_x[c] = x[c0 + c];
    for (int i = tid; i < cnt; i += FWD_T) s_y[i] = p.y[i];
    __syncthreads();
    V yv[RC];
#pragma unroll
    for (int r = 0; r < RC; ++r) {
        const int qq = g + G * r;
        yv[r] = (qq < cnt) ? (V)s_y[qq] : (V)0;
    }
    V pacc[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r) pacc[r] = (V)0;
    // the next sub-slab's rows in flight too while they fit the registers
    constexpr bool PF = MS && (RC + RN <= 11);
    constexpr int RPc = PF ? RC : 1, RPn = PF ? RN : 1;
    for (int64_t sub = c0; sub < c1; sub += SWC) {
        const int64_t col = sub + (int64_t)v * VW;
        const bool more = sub + SWC < c1;   // uniform
        uvec4 ua2[RPc], un2[RPn];
        if constexpr (PF) {
            if (more) {
                const int64_t coln = col + SWC;
#pragma unroll
                for (int r = 0; r < RC; ++r)
                    ua2[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, coln,
                                                 c1, crow[r] >= 0, A, c0);
#pragma unroll
                for (int r = 0; r < RN; ++r)
                    un2[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, coln,
                                                 c1, nrow[r] >= 0, A, c0);
            }
        } else if (sub != c0) {
#pragma unroll
            for (int r = 0; r < RC; ++r)
                ua[r] = load_raw_sel<T, AL>(A + (int64_t)(crow[r] >= 0 ? crow[r] : 0) * p.ld, col, c1,
                                            crow[r] >= 0, A, c0);
#pragma unroll
            for (int r = 0; r < RN; ++r)
                un[r] = load_raw_sel<T, AL>(A + (int64_t)(nrow[r] >= 0 ? nrow[r] : 0) * p.ld, col, c1,
                                            nrow[r] >= 0, A, c0);
        }
        if (cnt > 0) {   // uniform
            V acc[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = (V)0;
#pragma unroll
            for (int r = 0; r < RC; ++r) {
                V a[VW];
                cvt_raw<T, V>(ua[r], a);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc[e] = fmaT(a[e], yv[r], acc[e]);
            }
#pragma unroll
            for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
            __syncthreads();
            if (tid < SWC) {
                const int64_t cc = sub + tid;
                if (cc < c1) {
                    V s = (V)0;
                    for (int gg = 0; gg < G; ++gg) s += s_red[gg][tid];
                    s_x[cc - c0] += s;
                }
            }
            __syncthreads();
        }
        if (col < c1) {
#pragma unroll
            for (int r = 0; r < RN; ++r) {
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
                for (int r = 0; r < RC; ++r) ua[r] = ua2[r];
#pragma unroll
                for (int r = 0; r < RN; ++r) un[r] = un2[r];
            }
        }
    }
    if (cnt > 0)
        for (int c = tid; c < wcols; c += FWD_T) x[c0 + c] = s_x[c];
    if (ncnt == 0) return;   // uniform: the last iteration has no next products
    // each row's NV lane sums (consecutive lanes of one wave) by a fixed
    // butterfly
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        const V s = group_sum(pacc[r], NV);
        if (v == 0 && nrow[r] >= 0)
            p.Pout[(int64_t)blockIdx.x * 3 * p.bmax + nidx[r]] = (double)s;
    }
    // count this workgroup done; the last one sums the partials
    __shared__ int s_last;
    __syncthreads();
    if (tid == 0)
        s_last = (__hip_atomic_fetch_add(p.counter, 1u, __ATOMIC_ACQ_REL,
                                         __HIP_MEMORY_SCOPE_AGENT) == gridDim.x - 1) ? 1 : 0;
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (tid == 0) *p.counter = 0u;   // ready for the next launch
    // two threads per slot, each summing alternate chunks (all loads of a
    // batch in flight), then the pair's sum
    const V *__restrict__ bv = (const V *)p.b;
    const int slot = tid >> 1, h = tid & 1;
    if (slot < 3 * FWD_B) {
        const int l = slot / FWD_B, i = slot - l * FWD_B;
        const int cl = (l == 0) ? B.c0 : ((l == 1) ? B.c1 : B.c2);
        const bool ok = i < cl;
        const int64_t row = (l == 0 ? B.s0 : (l == 1 ? B.s1 : B.s2)) + (ok ? i : 0);
        const V bt = bv[row];
        const double *pp = p.Pout + (ok ? l * p.bmax + i : 0);
        const int64_t st = 3 * (int64_t)p.bmax;
        const int nch = gridDim.x;
        double acc = 0.0;
        int ch = h;
        for (; ch + 14 < nch; ch += 16) {
            const double t0 = pp[(int64_t)ch * st], t1 = pp[(int64_t)(ch + 2) * st];
            const double t2 = pp[(int64_t)(ch + 4) * st], t3 = pp[(int64_t)(ch + 6) * st];
            const double t4 = pp[(int64_t)(ch + 8) * st], t5 = pp[(int64_t)(ch + 10) * st];
            const double t6 = pp[(int64_t)(ch + 12) * st], t7 = pp[(int64_t)(ch + 14) * st];
            acc += t0; acc += t1; acc += t2; acc += t3;
            acc += t4; acc += t5; acc += t6; acc += t7;
        }
        for (; ch < nch; ch += 2) acc += pp[(int64_t)ch * st];
        const double o = __shfl_xor(acc, 1, 2);
        const double tot = h ? (o + acc) : (acc + o);
        if (h == 0) p.z3[slot] = ok ? (double)bt - tot : 0.0;
    }
}

// ---------------------------------------------------- three sampled steps --
// The inner loop of Algorithm 1 for outer iteration it: y1, y2, y3 from
// z = b_S - A_S x0 (formed by the last workgroup of the previous kernel), the
// stored inverses H1, H2, H3 and the cross-Grams xg ([3][bmax][bmax], see
// xgram_tile):
//   z_l = b_l - A_l x0;  y1 = H1 z1;  z2 -= G21 y1;  z3 -= G31 y1;
//   y2 = H2 z2;  z3 -= G32 y2;  y3 = H3 z3;
// every workgroup forms the same y (same order), then updates its column slab
// x[cols] += A_S[:, cols]^T y over the rows of all three blocks.
//
// Memory round trips: the draws, then everything else at once.  Thread range
// k = 0, 1, 2 (2 FWD_B threads each) reads H1, G21, G31 into registers
// (thread u of a range takes row u / 2 and columns (u % 2) + 2 t); every
// thread reads its share of H2, G32, H3, which go to LDS once the first two
// stages are done; every thread also loads its entries of x and z, and its
// rows of the update once the registers of the first half are free.  Each
// stage of the chain is then register or LDS work, a shuffle and a barrier.
// Chain form (K > 0): the previous iteration's greedy rows I with their y
// join the update, x += A_I^T y_I + sum_l A_l^T y_l, in the same pass (z then
// already accounts for the greedy step, see k_gram_chain).
struct FwdSamp3P {
    const void *A;
    int64_t ld, n, q, rem;
    int bmax;
    const int32_t *tau;
    int64_t tau_index;
    const double *H;
    const double *xg;
    const double *z3;      // z of the three blocks, slots l * FWD_B + i
    void *x;
    int64_t wu;
    const Ctrl *ctrl;
    const int32_t *I;      // chain form: the greedy rows of the previous iteration
    int K;                 // (0: none) and their y, applied in the same pass
    const double *y;
};

constexpr int MC = (FWD_B + 1) / 2;          // matrix entries per thread and row pair
constexpr int LDM = FWD_B;                   // row stride of the matrices kept in LDS
constexpr int FILL = (3 * FWD_B * FWD_B + FWD_T - 1) / FWD_T;   // LDS entries per thread

// Entry (i, j) of a matrix stored at M[i * si + j * sj] into m[t] for
// j = h + 2 t, zero outside rows x cols; every load reads an in-bounds
// address (entry (0, 0) stands in) so that none sits behind a branch.
__device__ __forceinline__ void mv_load(const double *__restrict__ M, int64_t si, int64_t sj,
                                        int i, int h, int rows, int cols, double (&m)[MC]) {
    const bool okr = i < rows;
#pragma unroll
    for (int t = 0; t < MC; ++t) {
        const int j = h + 2 * t;
        const bool ok = okr && j < cols;
        const double v = M[ok ? (int64_t)i * si + (int64_t)j * sj : 0];
        m[t] = ok ? v : 0.0;
    }
}

// sum_j m[t] vin[h + 2 t] over the pair of threads: four accumulators in a
// fixed order, then the pair's sum.  Entries past the matrix are zero in m,
// and vin holds finite values at every index read (h + 2 t < FWD_B + 1 is
// clamped).
__device__ __forceinline__ double mv_dot(const double (&m)[MC], const double *vin, int h) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
#pragma unroll
    for (int t = 0; t < MC; t += 4) {
        a0 = __builtin_fma(m[t], vin[(h + 2 * t) < FWD_B ? h + 2 * t : 0], a0);
        if (t + 1 < MC) a1 = __builtin_fma(m[t + 1], vin[h + 2 * t + 2], a1);
        if (t + 2 < MC) a2 = __builtin_fma(m[t + 2], vin[h + 2 * t + 4], a2);
        if (t + 3 < MC) a3 = __builtin_fma(m[t + 3], vin[h + 2 * t + 6], a3);
    }
    const double s = (a0 + a1) + (a2 + a3);
    const double o = __shfl_xor(s, 1, 2);
    return h ? (o + s) : (s + o);
}

// The same product with the matrix row in LDS (L[i * LDM + j], zero outside
// the matrix; a column index past the row, h + 2 t = FWD_B, contributes 0).
__device__ __forceinline__ double mv_dot_lds(const double *L, int i, const double *vin, int h) {
    double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
    const double *Lr = L + (i < FWD_B ? i : 0) * LDM;
#pragma unroll
    for (int t = 0; t < MC; t += 4) {
        const int j0 = h + 2 * t;
        const bool in = j0 < FWD_B;
        const double lv = Lr[in ? j0 : 0];
        a0 = __builtin_fma(in ? lv : 0.0, vin[in ? j0 : 0], a0);
        if (t + 1 < MC) a1 = __builtin_fma(Lr[j0 + 2], vin[j0 + 2], a1);
        if (t + 2 < MC) a2 = __builtin_fma(Lr[j0 + 4], vin[j0 + 4], a2);
        if (t + 3 < MC) a3 = __builtin_fma(Lr[j0 + 6], vin[j0 + 6], a3);
    }
    const double s = (a0 + a1) + (a2 + a3);
    const double o = __shfl_xor(s, 1, 2);
    return h ? (o + s) : (s + o);
}

template <typename T, typename V, bool AL, int RN, bool MS>
__global__ __launch_bounds__(FWD_T) void k_fwd_samp3(FwdSamp3P p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int SWC = fwd_swc<T>();
    constexpr int NV = SWC / VW;
    constexpr int G = FWD_T / NV;
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;
    Blk3 B;
    blocks3(p.tau, p.tau_index, p.q, p.rem, B);
    const int64_t hoff0 = blk_hoff(p.tau[p.tau_index], p.q, p.rem);
    const int64_t hoff1 = blk_hoff(p.tau[p.tau_index + 1], p.q, p.rem);
    const int64_t hoff2 = blk_hoff(p.tau[p.tau_index + 2], p.q, p.rem);
    const int ncnt = B.c0 + B.c1 + B.c2;
    const int bm = p.bmax;
    const int n0 = B.c0, n1 = B.c1, n2 = B.c2;
    if (p.ctrl->done) return;
    const int64_t c0 = (int64_t)blockIdx.x * p.wu;
    const int64_t c1 = (c0 + p.wu < p.n) ? c0 + p.wu : p.n;
    const int wcols = (int)(c1 - c0);

    __shared__ V s_x[1024];
    __shared__ V s_red[G][SWC];
    __shared__ double s_z[3 * FWD_B], s_y[3 * FWD_B + 64];
    __shared__ double s_m[3 * FWD_B * LDM];
    static_assert(64 + 3 * FWD_B <= FWD_T, "one row-table entry per thread");
    __shared__ int32_t s_row[64 + 3 * FWD_B], s_slot[64 + 3 * FWD_B];
    const int K = p.K;

    // --- every load of the kernel, in the order the data is needed
    V xv[(1024 + FWD_T - 1) / FWD_T];
#pragma unroll
    for (int u = 0; u < (1024 + FWD_T - 1) / FWD_T; ++u) {
        const int c = tid + u * FWD_T;
        const V t = x[c0 + (c < wcols ? c : 0)];
        xv[u] = (c < wcols) ? t : (V)0;
    }
    const double zv = p.z3[tid < 3 * FWD_B ? tid : 0];
    // chain form: the greedy rows and their y (uniform branch)
    int32_t iv = 0;
    double ygv = 0.0;
    if (K > 0) {
        iv = p.I[tid < K ? tid : 0];
        ygv = p.y[tid < K ? tid : 0];
    }
    // the first three matrices of the chain, one per thread range
    const int rg = tid / (2 * FWD_B), uu = tid - rg * 2 * FWD_B, ir = uu >> 1, h = uu & 1;
    double m[MC];
    {
        const double *M = p.H;
        int64_t sj = 1;
        int rows = 0, cols = 0;
        if (rg == 0) { M = p.H + hoff0; sj = n0; rows = n0; cols = n0; }   // H1 read transposed
        else if (rg == 1) { M = p.xg; sj = bm; rows = n1; cols = n0; }     // G21, column-major
        else if (rg == 2) { M = p.xg + (int64_t)bm * bm; sj = bm; rows = n2; cols = n0; }   // G31
        mv_load(M, 1, sj, ir, h, rows, cols, m);
    }
    // this thread's share of H2, G32, H3 (for LDS), zero outside each matrix;
    // consecutive threads take consecutive i, i.e. consecutive addresses
    double fv[FILL];
#pragma unroll
    for (int u = 0; u < FILL; ++u) {
        const int e = tid + u * FWD_T;
        const int k = e / (FWD_B * FWD_B), rr = e - k * FWD_B * FWD_B;
        const int j = rr / FWD_B, i = rr - j * FWD_B;    // LDS position (i, j)
        const double *M = (k == 0) ? p.H + hoff1 : ((k == 1) ? p.xg + 2 * (int64_t)bm * bm : p.H + hoff2);
        const int rows = (k == 0) ? n1 : n2, cols = (k == 1) ? n1 : (k == 0 ? n1 : n2);
        const int64_t sj = (k == 1) ? bm : (k == 0 ? n1 : n2);
        const bool ok = k < 3 && i < rows && j < cols;
        const double t = M[ok ? i + (int64_t)j * sj : 0];
        fv[u] = ok ? t : 0.0;
    }
    // row r of this thread's share of the update: its index in A (row 0
    // stands in past the last row) and its slot in s_y, read from the LDS
    // tables each time it is needed (volatile: not held in registers across
    // the chain).  The greedy rows come first.
    const int nrows = K + ncnt;
    auto urow = [&](int r, int64_t *row, int *slot) -> bool {
        const int qq = g + G * r;
        const bool ok = qq < nrows;
        *row = ok ? (int64_t)((volatile int32_t *)s_row)[qq] : 0;
        *slot = ok ? ((volatile int32_t *)s_slot)[qq] : 0;
        return ok;
    };

    // --- z = b_S - A_S x0 (slots l * FWD_B + i; s_y zeroed)
#pragma unroll
    for (int u = 0; u < (1024 + FWD_T - 1) / FWD_T; ++u) {
        const int c = tid + u * FWD_T;
        if (c < wcols) s_x[c] = xv[u];
    }
    if (tid < 3 * FWD_B) {
        s_z[tid] = zv;
        s_y[tid] = 0.0;
    }
    if (tid < K) s_y[3 * FWD_B + tid] = ygv;
    // the row tables of the update: entry tid (fewer than FWD_T rows)
    if (tid < nrows) {
        int l, i;
        int64_t r3;
        split3(B, tid >= K ? tid - K : 0, &l, &i, &r3);
        s_row[tid] = (tid < K) ? iv : (int32_t)r3;
        s_slot[tid] = (tid < K) ? 3 * FWD_B + tid : l * FWD_B + i;
    }
    __syncthreads();
    // y1 = H1 z1
    if (rg == 0) {
        const double d = mv_dot(m, s_z, h);
        if (h == 0 && ir < n0) s_y[ir] = d;
    }
    __syncthreads();
    // z2 -= G21 y1 and z3 -= G31 y1
    if (rg == 1 || rg == 2) {
        const double d = mv_dot(m, s_y, h);
        const int rows = (rg == 1) ? n1 : n2;
        if (h == 0 && ir < rows) s_z[rg * FWD_B + ir] -= d;
    }
    // the second half of the chain's matrices into LDS
#pragma unroll
    for (int u = 0; u < FILL; ++u) {
        const int e = tid + u * FWD_T;
        if (e < 3 * FWD_B * FWD_B) {
            const int k = e / (FWD_B * FWD_B), rr = e - k * FWD_B * FWD_B;
            const int j = rr / FWD_B, i = rr - j * FWD_B;
            s_m[k * FWD_B * LDM + i * LDM + j] = fv[u];
        }
    }
    // the rows of the update (first sub-slab) load during the rest of the
    // chain, once the registers of the first half are free
    uvec4 ua[RN];
    {
        const int64_t col = c0 + (int64_t)v * VW;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            int64_t row;
            int slot;
            const bool ok = urow(r, &row, &slot);
            ua[r] = load_raw_sel<T, AL>(A + row * p.ld, col, c1, ok, A, c0);
        }
    }
    __syncthreads();
    // y2 = H2 z2
    if (rg == 0) {
        const double d = mv_dot_lds(s_m, ir, s_z + FWD_B, h);
        if (h == 0 && ir < n1) s_y[FWD_B + ir] = d;
    }
    __syncthreads();
    // z3 -= G32 y2
    if (rg == 1) {
        const double d = mv_dot_lds(s_m + FWD_B * LDM, ir, s_y + FWD_B, h);
        if (h == 0 && ir < n2) s_z[2 * FWD_B + ir] -= d;
    }
    __syncthreads();
    // y3 = H3 z3
    if (rg == 2) {
        const double d = mv_dot_lds(s_m + 2 * FWD_B * LDM, ir, s_z + 2 * FWD_B, h);
        if (h == 0 && ir < n2) s_y[2 * FWD_B + ir] = d;
    }
    __syncthreads();

    // --- x[cols] += A_S[:, cols]^T y
    V yv[RN];
#pragma unroll
    for (int r = 0; r < RN; ++r) {
        int64_t row;
        int slot;
        const bool ok = urow(r, &row, &slot);
        yv[r] = ok ? (V)s_y[slot] : (V)0;
    }
    constexpr bool PF = MS && RN <= 5;
    constexpr int RP = PF ? RN : 1;
    for (int64_t sub = c0; sub < c1; sub += SWC) {
        const int64_t col = sub + (int64_t)v * VW;
        const bool more = sub + SWC < c1;   // uniform
        uvec4 ua2[RP];
        if constexpr (PF) {
            if (more) {
                const int64_t coln = col + SWC;
#pragma unroll
                for (int r = 0; r < RN; ++r) {
                    int64_t row;
                    int slot;
                    const bool ok = urow(r, &row, &slot);
                    ua2[r] = load_raw_sel<T, AL>(A + row * p.ld, coln, c1, ok, A, c0);
                }
            }
        } else if (sub != c0) {
#pragma unroll
            for (int r = 0; r < RN; ++r) {
                int64_t row;
                int slot;
                const bool ok = urow(r, &row, &slot);
                ua[r] = load_raw_sel<T, AL>(A + row * p.ld, col, c1, ok, A, c0);
            }
        }
        V acc[VW];
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = (V)0;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            V a[VW];
            cvt_raw<T, V>(ua[r], a);
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = fmaT(a[e], yv[r], acc[e]);
        }
#pragma unroll
        for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
        __syncthreads();
        if (tid < SWC) {
            const int64_t cc = sub + tid;
            if (cc < c1) {
                V s = (V)0;
                for (int gg = 0; gg < G; ++gg) s += s_red[gg][tid];
                s_x[cc - c0] += s;
            }
        }
        __syncthreads();
        if constexpr (PF) {
            if (more) {
#pragma unroll
                for (int r = 0; r < RN; ++r) ua[r] = ua2[r];
            }
        }
    }
    for (int c = tid; c < wcols; c += FWD_T) x[c0 + c] = s_x[c];
}

// ------------------------------------------------------- chain step kernel --
// The rest of iteration it after the chain form's Grams (k_gram_chain), in one
// launch over the column slabs (one sub-slab each): in every workgroup wave 0
// solves the greedy system (G + lambda I) y = r_I (ldl_blk64 on the summed
// Gram chunks; every workgroup forms the same y) while waves 1-7 sum C into
// LDS and load the three sampled steps' matrices into registers, so that their
// memory latency is spent during the factorisation.  Then
// z = r_{S'} - C y (j ascending), the chain of k_fwd_samp3 with the same
// arithmetic (the same thread of a row pair, the same sums), and
// x[cols] += A_I[:, cols]^T y + sum_l A_l[:, cols]^T y_l in one pass.  The
// first workgroup writes y and, for a checkpoint, the chain state (I, y, z).
struct FwdChainP {
    const void *A;
    int64_t ld, n, q, rem;
    int bmax;
    const int32_t *tau;
    int64_t tau_index;     // first draw of iteration it + 1
    const double *H;
    const double *xg;      // cross-Grams of iteration it + 1's blocks
    const double *G;       // [nch][K (K + 1) / 2] packed lower partials
    const double *C;       // [nch][3 * FWD_B][64] partials
    int nch;
    int K;
    double lambda;
    const double *rI;
    const void *r;         // residual of iteration it (vector type)
    const int32_t *I;
    void *x;
    int64_t wu;            // columns per workgroup (one sub-slab)
    double *y;
    double *ckst;          // NULL, or a checkpoint's chain state
    Ctrl *ctrl;
};

constexpr int CHN = 4;                       // most column chunks of G and C
constexpr int FC_T = FWD_T - 64;             // threads of waves 1-7
constexpr int FILL2 = (3 * FWD_B * FWD_B + FC_T - 1) / FC_T;   // H2, G32, H3 entries per thread
constexpr int LA = 64 * 65 + 2 * 64;                          // LDS doubles: work matrix | colbuf

template <typename T, typename V, bool AL, int RN>
__global__ __launch_bounds__(FWD_T) void k_fwd_chain(FwdChainP p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int SWC = fwd_swc<T>();
    constexpr int NV = SWC / VW;
    constexpr int G = FWD_T / NV;
    static_assert(1024 + G * SWC * sizeof(V) / 8 <= LA, "phase-2 arrays fit the factorisation's LDS");
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const int tid = threadIdx.x;
    const int K = p.K, KP = K * (K + 1) / 2;
    // LDS: region a holds the factorisation (the padded system, then L; column buffers),
    // then z, y and the update's row sums; region b holds C, then H2, G32, H3
    __shared__ double lds_a[LA];
    __shared__ double lds_b[3 * FWD_B * LDM];
    __shared__ double s_yk[64], s_rs[3 * FWD_B];
    __shared__ int32_t s_rok[3 * FWD_B];
    __shared__ V s_x[SWC];
    __shared__ int32_t s_row[64 + 3 * FWD_B], s_slot[64 + 3 * FWD_B];
    __shared__ int s_ok;
    double *Lc = lds_a, *colbuf = Lc + 64 * 65;
    double *s_z = lds_a, *s_y = lds_a + 256;
    V (*s_red)[SWC] = reinterpret_cast<V (*)[SWC]>(lds_a + 1024);

    // --- phase 0: the Gram chunks (summed in chunk order) and r_I
    constexpr int NU0 = (64 * 65 / 2 + FWD_T - 1) / FWD_T;
    {
        const int stop =
            __hip_atomic_load(&p.ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        double gt[CHN][NU0];
#pragma unroll
        for (int c = 0; c < CHN; ++c)
#pragma unroll
            for (int u = 0; u < NU0; ++u) {
                const int f = tid + u * FWD_T;
                gt[c][u] = p.G[(int64_t)(c < p.nch ? c : 0) * KP + (f < KP ? f : 0)];
            }
        const double ri = p.rI[tid < K ? tid : 0];
        if (stop) return;
        // the padded system straight into the work matrix (lambda on the
        // diagonal, the identity beyond K)
#pragma unroll
        for (int u = 0; u < NU0; ++u) {
            const int f = tid + u * FWD_T;
            double gs = gt[0][u];
#pragma unroll
            for (int c = 1; c < CHN; ++c) gs += (c < p.nch) ? gt[c][u] : 0.0;
            if (f < 64 * 65 / 2) lb_put(Lc, f, gs, K, p.lambda);
        }
        if (tid < 64) s_yk[tid] = (tid < K) ? ri : 0.0;
    }
    __syncthreads();

    // --- phase 1: wave 0 factors (nothing else is live across it; the
    // wave index is made scalar so that both branches are real jumps) ...
    const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
    if (wv == 0) {
        const bool ok = ldl_blk64(Lc, s_yk, K, colbuf);
        if (tid == 0) {
            s_ok = ok ? 1 : 0;
            if (!ok) {
                p.ctrl->status = RORBK_ERR_NOT_SPD;
                p.ctrl->done = 1;
            }
        }
    }
    // ... while waves 1-7 load everything else
    double m[MC];
    double fv[FILL2];
    if (wv != 0) {
        const int t = tid - 64;
        const int rg = t / (2 * FWD_B), uu = t - rg * 2 * FWD_B, ir = uu >> 1, h = uu & 1;
        Blk3 B;
        blocks3(p.tau, p.tau_index, p.q, p.rem, B);
        const int64_t hoff0 = blk_hoff(p.tau[p.tau_index], p.q, p.rem);
        const int64_t hoff1 = blk_hoff(p.tau[p.tau_index + 1], p.q, p.rem);
        const int64_t hoff2 = blk_hoff(p.tau[p.tau_index + 2], p.q, p.rem);
        const int ncnt = B.c0 + B.c1 + B.c2, nrows = K + ncnt;
        const int bm = p.bmax, n0 = B.c0, n1 = B.c1, n2 = B.c2;
        const int64_t c0 = (int64_t)blockIdx.x * p.wu;
        const int wcols = (int)(((c0 + p.wu < p.n) ? c0 + p.wu : p.n) - c0);
        // r at the next blocks' rows, the greedy rows, the slab of x
        double rsv = 0.0;
        int rok = 0;
        if (t < 3 * FWD_B) {
            const int l = t / FWD_B, i = t - l * FWD_B;
            const int cl = (l == 0) ? n0 : ((l == 1) ? n1 : n2);
            const int64_t st = (l == 0) ? B.s0 : ((l == 1) ? B.s1 : B.s2);
            rok = i < cl;
            const V rr = ((const V *)p.r)[st + (rok ? i : 0)];
            rsv = rok ? (double)rr : 0.0;
        }
        const int32_t iv = p.I[t < K ? t : 0];
        const V xv = x[c0 + (t < wcols ? t : 0)];
        // H1, G21, G31 (thread ranges of 2 FWD_B, as k_fwd_samp3)
        {
            const double *M = p.H;
            int64_t sj = 1;
            int rows = 0, cols = 0;
            if (rg == 0) { M = p.H + hoff0; sj = n0; rows = n0; cols = n0; }
            else if (rg == 1) { M = p.xg; sj = bm; rows = n1; cols = n0; }
            else if (rg == 2) { M = p.xg + (int64_t)bm * bm; sj = bm; rows = n2; cols = n0; }
            mv_load(M, 1, sj, ir, h, rows, cols, m);
        }
        // H2, G32, H3 for LDS (consecutive threads, consecutive addresses)
#pragma unroll
        for (int u = 0; u < FILL2; ++u) {
            const int e = t + u * FC_T;
            const int k = e / (FWD_B * FWD_B), rr = e - k * FWD_B * FWD_B;
            const int j = rr / FWD_B, i = rr - j * FWD_B;
            const double *M = (k == 0) ? p.H + hoff1 : ((k == 1) ? p.xg + 2 * (int64_t)bm * bm : p.H + hoff2);
            const int rows = (k == 0) ? n1 : n2, cols = (k == 1) ? n1 : (k == 0 ? n1 : n2);
            const int64_t sj = (k == 1) ? bm : (k == 0 ? n1 : n2);
            const bool ok = k < 3 && i < rows && j < cols;
            const double tv = M[ok ? i + (int64_t)j * sj : 0];
            fv[u] = ok ? tv : 0.0;
        }
        if (t < 3 * FWD_B) {
            s_rs[t] = rsv;
            s_rok[t] = rok;
        }
        if (t < wcols) s_x[t] = xv;
        if (t < nrows) {   // the update's row tables, greedy rows first
            int l, i;
            int64_t r3;
            split3(B, t >= K ? t - K : 0, &l, &i, &r3);
            s_row[t] = (t < K) ? iv : (int32_t)r3;
            s_slot[t] = (t < K) ? 3 * FWD_B + t : l * FWD_B + i;
        }
        // C summed over its chunks into LDS (row stride LDM), in batches
        constexpr int NCE = 3 * FWD_B * 64, PT = (NCE + FC_T - 1) / FC_T, UB = 7;
        for (int ub = 0; ub < PT; ub += UB) {
            double ct[CHN][UB];
#pragma unroll
            for (int c = 0; c < CHN; ++c)
#pragma unroll
                for (int u = 0; u < UB; ++u) {
                    const int e = t + (ub + u) * FC_T;
                    ct[c][u] = p.C[(int64_t)(c < p.nch ? c : 0) * NCE + (e < NCE ? e : 0)];
                }
#pragma unroll
            for (int u = 0; u < UB; ++u) {
                const int e = t + (ub + u) * FC_T;
                double cs = ct[0][u];
#pragma unroll
                for (int c = 1; c < CHN; ++c) cs += (c < p.nch) ? ct[c][u] : 0.0;
                const int sl = e >> 6, j = e & 63;
                if (e < NCE) lds_b[sl * LDM + j] = (j < K) ? cs : 0.0;
            }
        }
    }
    __syncthreads();
    if (!s_ok) return;

    // --- phase 2: z = r_{S'} - C y, then the chain (the sizes again, from
    // the draws)
    Blk3 B;
    blocks3(p.tau, p.tau_index, p.q, p.rem, B);
    const int ncnt = B.c0 + B.c1 + B.c2, nrows = K + ncnt;
    const int n0 = B.c0, n1 = B.c1, n2 = B.c2;
    const int64_t c0 = (int64_t)blockIdx.x * p.wu;
    const int64_t c1 = (c0 + p.wu < p.n) ? c0 + p.wu : p.n;
    const int wcols = (int)(c1 - c0);
    const int t = tid - 64;
    const int rg = t / (2 * FWD_B), uu = t - rg * 2 * FWD_B, ir = uu >> 1, h = uu & 1;
    const int g = tid / NV, v = tid % NV;
    if (tid < 3 * FWD_B) {
        double acc = 0.0;
        const double *cr = lds_b + tid * LDM;
        for (int j = 0; j < K; ++j) acc = __builtin_fma(cr[j], s_yk[j], acc);
        const double zz = s_rok[tid] ? s_rs[tid] - acc : 0.0;
        s_z[tid] = zz;
        s_y[tid] = 0.0;
        if (blockIdx.x == 0 && p.ckst) p.ckst[96 + tid] = zz;
    }
    if (tid < K) {
        s_y[3 * FWD_B + tid] = s_yk[tid];
        if (blockIdx.x == 0) {
            p.y[tid] = s_yk[tid];
            if (p.ckst) {
                reinterpret_cast<int32_t *>(p.ckst)[tid] = s_row[tid];
                p.ckst[32 + tid] = s_yk[tid];
            }
        }
    }
    __syncthreads();
    // H2, G32, H3 into LDS (C is no longer needed); y1 = H1 z1
    if (wv != 0) {
#pragma unroll
        for (int u = 0; u < FILL2; ++u) {
            const int e = t + u * FC_T;
            if (e < 3 * FWD_B * FWD_B) {
                const int k = e / (FWD_B * FWD_B), rr = e - k * FWD_B * FWD_B;
                const int j = rr / FWD_B, i = rr - j * FWD_B;
                lds_b[k * FWD_B * LDM + i * LDM + j] = fv[u];
            }
        }
        if (rg == 0) {
            const double d = mv_dot(m, s_z, h);
            if (h == 0 && ir < n0) s_y[ir] = d;
        }
    }
    __syncthreads();
    // z2 -= G21 y1 and z3 -= G31 y1
    if (wv != 0 && (rg == 1 || rg == 2)) {
        const double d = mv_dot(m, s_y, h);
        const int rows = (rg == 1) ? n1 : n2;
        if (h == 0 && ir < rows) s_z[rg * FWD_B + ir] -= d;
    }
    // the update's rows load during the rest of the chain
    const int64_t col = c0 + (int64_t)v * VW;
    uvec4 ua[RN];
    {
        // every row index first (LDS), then every load, so that the loads
        // do not wait on one LDS read each
        int32_t rw[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int qq = g + G * r;
            rw[r] = (qq < nrows) ? s_row[qq] : 0;
        }
#pragma unroll
        for (int r = 0; r < RN; ++r)
            ua[r] = load_raw_sel<T, AL>(A + (int64_t)rw[r] * p.ld, col, c1, g + G * r < nrows, A,
                                        c0);
    }
    __syncthreads();
    // y2 = H2 z2
    if (wv != 0 && rg == 0) {
        const double d = mv_dot_lds(lds_b, ir, s_z + FWD_B, h);
        if (h == 0 && ir < n1) s_y[FWD_B + ir] = d;
    }
    __syncthreads();
    // z3 -= G32 y2
    if (wv != 0 && rg == 1) {
        const double d = mv_dot_lds(lds_b + FWD_B * LDM, ir, s_y + FWD_B, h);
        if (h == 0 && ir < n2) s_z[2 * FWD_B + ir] -= d;
    }
    __syncthreads();
    // y3 = H3 z3
    if (wv != 0 && rg == 2) {
        const double d = mv_dot_lds(lds_b + 2 * FWD_B * LDM, ir, s_z + 2 * FWD_B, h);
        if (h == 0 && ir < n2) s_y[2 * FWD_B + ir] = d;
    }
    __syncthreads();

    // --- x[cols] += A_I^T y + sum_l A_l^T y_l (one sub-slab)
    V acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = (V)0;
    {
        // the slots, then their y, then the products (no LDS read waits on
        // another inside the loop)
        int32_t sl[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            const int qq = g + G * r;
            sl[r] = (qq < nrows) ? s_slot[qq] : -1;
        }
        V yv[RN];
#pragma unroll
        for (int r = 0; r < RN; ++r) yv[r] = (sl[r] >= 0) ? (V)s_y[sl[r] >= 0 ? sl[r] : 0] : (V)0;
#pragma unroll
        for (int r = 0; r < RN; ++r) {
            V av[VW];
            cvt_raw<T, V>(ua[r], av);
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = fmaT(av[e], yv[r], acc[e]);
        }
    }
#pragma unroll
    for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
    __syncthreads();
    if (tid < wcols) {
        V sx = (V)0;
        for (int gg = 0; gg < G; ++gg) sx += s_red[gg][tid];
        x[c0 + tid] = s_x[tid] + sx;
    }
}

// ------------------------------------------------------------ launchers --
// Size class of the per-thread row counts: rows of one block (RC) and of
// three (RN) per thread for G row groups.
template <typename T>
constexpr int fwd_groups() { return FWD_T / (fwd_swc<T>() / Tr<T>::VW); }

static int fwd_class(int bmax, int G) {
    const int rc = (bmax + G - 1) / G, rn = (3 * bmax + G - 1) / G;
    if (rc <= 2 && rn <= 4) return 0;
    if (rc <= 3 && rn <= 8) return 1;
    return 2;   // rc <= 5, rn <= 13: FWD_B = 65 rows over 16 or 32 row groups
}

template <typename T, typename V, bool AL, bool MS>
static hipError_t greedy_launch_cls(const FwdGreedyP &p, int nblk, int cls, hipStream_t s) {
    switch (cls) {
    case 0: hipLaunchKernelGGL((k_fwd_greedy<T, V, AL, 2, 4, MS>), dim3(nblk), dim3(FWD_T), 0, s, p); break;
    case 1: hipLaunchKernelGGL((k_fwd_greedy<T, V, AL, 3, 8, MS>), dim3(nblk), dim3(FWD_T), 0, s, p); break;
    default: hipLaunchKernelGGL((k_fwd_greedy<T, V, AL, 5, 13, MS>), dim3(nblk), dim3(FWD_T), 0, s, p); break;
    }
    return hipGetLastError();
}

// rows of the update per thread (the three blocks and, in the chain form,
// the greedy rows): 4, 8, 13 or 17
template <typename T, typename V, bool AL, bool MS>
static hipError_t samp3_launch_rn(const FwdSamp3P &p, int nblk, int bmax, hipStream_t s) {
    constexpr int G = fwd_groups<T>();
    const int rn = (3 * bmax + p.K + G - 1) / G;
    if (rn <= 4)
        hipLaunchKernelGGL((k_fwd_samp3<T, V, AL, 4, MS>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else if (rn <= 8)
        hipLaunchKernelGGL((k_fwd_samp3<T, V, AL, 8, MS>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else if (rn <= 13)
        hipLaunchKernelGGL((k_fwd_samp3<T, V, AL, 13, MS>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else
        hipLaunchKernelGGL((k_fwd_samp3<T, V, AL, 17, MS>), dim3(nblk), dim3(FWD_T), 0, s, p);
    return hipGetLastError();
}

template <typename T, typename V>
static hipError_t fwd_greedy_typed(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    FwdGreedyP p;
    p.A = a.A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.bmax = (int)L.bmax;
    p.tau = h->d_tau;
    p.tau_next = a.tau_index;
    p.I = a.I;
    p.K = (int)L.K;
    p.y = a.y;
    p.x = a.x;
    p.Pout = h->d_P3;
    p.wu = L.wf;
    p.ctrl = h->d_ctrl;
    p.b = a.b;
    p.z3 = h->d_z3;
    p.counter = h->d_fwdcnt;
    const int cls = fwd_class((int)L.bmax, fwd_groups<T>());
    const bool ms = L.wf > fwd_swc<T>();
    if (a.aligned) {
        if (ms) return greedy_launch_cls<T, V, true, true>(p, L.nch_f, cls, s);
        return greedy_launch_cls<T, V, true, false>(p, L.nch_f, cls, s);
    }
    if (ms) return greedy_launch_cls<T, V, false, true>(p, L.nch_f, cls, s);
    return greedy_launch_cls<T, V, false, false>(p, L.nch_f, cls, s);
}

template <typename T, typename V>
static hipError_t fwd_samp3_typed(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    FwdSamp3P p;
    p.A = a.A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.bmax = (int)L.bmax;
    p.tau = h->d_tau;
    p.tau_index = a.tau_index;
    p.H = h->d_H;
    p.xg = a.xg;
    p.z3 = h->d_z3;
    p.x = a.x;
    p.wu = L.wf;
    p.ctrl = h->d_ctrl;
    p.I = a.I;
    p.K = a.I ? (int)L.K : 0;
    p.y = a.y;
    const int bm = (int)L.bmax;
    const bool ms = L.wf > fwd_swc<T>();
    if (a.aligned) {
        if (ms) return samp3_launch_rn<T, V, true, true>(p, L.nch_f, bm, s);
        return samp3_launch_rn<T, V, true, false>(p, L.nch_f, bm, s);
    }
    if (ms) return samp3_launch_rn<T, V, false, true>(p, L.nch_f, bm, s);
    return samp3_launch_rn<T, V, false, false>(p, L.nch_f, bm, s);
}

hipError_t launch_fwd_greedy(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s) {
    if (a.vec == VEC_F64) return fwd_greedy_typed<double, double>(h, a, s);
    if (a.dt == RORBK_F32) return fwd_greedy_typed<float, float>(h, a, s);
    return fwd_greedy_typed<bf16_t, float>(h, a, s);
}

hipError_t launch_fwd_samp3(const rorbk_handle_s *h, const FwdArgs &a, hipStream_t s) {
    if (a.vec == VEC_F64) return fwd_samp3_typed<double, double>(h, a, s);
    if (a.dt == RORBK_F32) return fwd_samp3_typed<float, float>(h, a, s);
    return fwd_samp3_typed<bf16_t, float>(h, a, s);
}

template <typename T, int NW>
static hipError_t xgram_typed(const rorbk_handle_s *h, const void *A, int aligned, int64_t ti,
                              double *out, hipStream_t s) {
    const Layout &L = h->L;
    const int jobs = xgram_jobs((int)L.bmax);
    if (aligned)
        hipLaunchKernelGGL((k_xgram<T, true, NW>), dim3(jobs), dim3(64 * NW), 0, s, (const T *)A,
                           L.ld, L.n, h->d_tau, ti, L.q, L.rem, (int)L.bmax, out,
                           (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_xgram<T, false, NW>), dim3(jobs), dim3(64 * NW), 0, s,
                           (const T *)A, L.ld, L.n, h->d_tau, ti, L.q, L.rem, (int)L.bmax, out,
                           (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

// waves: 4 (stand-alone starts, the residual's spare workgroups) or 8 (the
// selection's spare workgroups; the same sums when a chained solve resumes)
hipError_t launch_xgram(const rorbk_handle_s *h, const void *A, int dt, int aligned, int64_t ti,
                        double *out, int waves, hipStream_t s) {
    if (waves == 8) {
        if (dt == RORBK_F64) return xgram_typed<double, 8>(h, A, aligned, ti, out, s);
        if (dt == RORBK_F32) return xgram_typed<float, 8>(h, A, aligned, ti, out, s);
        return xgram_typed<bf16_t, 8>(h, A, aligned, ti, out, s);
    }
    if (dt == RORBK_F64) return xgram_typed<double, 4>(h, A, aligned, ti, out, s);
    if (dt == RORBK_F32) return xgram_typed<float, 4>(h, A, aligned, ti, out, s);
    return xgram_typed<bf16_t, 4>(h, A, aligned, ti, out, s);
}

int fwd_xgram_jobs(int bmax) { return xgram_jobs(bmax); }

template <typename T, typename V, bool AL>
static hipError_t fwd_chain_rn(const FwdChainP &p, int nblk, hipStream_t s) {
    constexpr int G = fwd_groups<T>();
    const int rn = (3 * p.bmax + p.K + G - 1) / G;
    if (rn <= 4)
        hipLaunchKernelGGL((k_fwd_chain<T, V, AL, 4>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else if (rn <= 8)
        hipLaunchKernelGGL((k_fwd_chain<T, V, AL, 8>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else if (rn <= 13)
        hipLaunchKernelGGL((k_fwd_chain<T, V, AL, 13>), dim3(nblk), dim3(FWD_T), 0, s, p);
    else
        hipLaunchKernelGGL((k_fwd_chain<T, V, AL, 17>), dim3(nblk), dim3(FWD_T), 0, s, p);
    return hipGetLastError();
}

template <typename T, typename V>
static hipError_t fwd_chain_typed(const rorbk_handle_s *h, const FwdArgs &a, const void *r,
                                  double *ckst, hipStream_t s) {
    const Layout &L = h->L;
    if (L.wf != fwd_swc<T>() || L.K > 64 || L.bmax > FWD_B || L.nch_c < 1 || L.nch_c > CHN)
        return hipErrorInvalidValue;   // one sub-slab per workgroup, the chain form's sizes
    FwdChainP p;
    p.A = a.A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.bmax = (int)L.bmax;
    p.tau = h->d_tau;
    p.tau_index = a.tau_index;
    p.H = h->d_H;
    p.xg = a.xg;
    p.G = h->d_G;
    p.C = h->d_C;
    p.nch = L.nch_c;
    p.K = (int)L.K;
    p.lambda = h->lambda;
    p.rI = h->d_rI;
    p.r = r;
    p.I = a.I;
    p.x = a.x;
    p.wu = L.wf;
    p.y = h->d_y;
    p.ckst = ckst;
    p.ctrl = h->d_ctrl;
    if (a.aligned) return fwd_chain_rn<T, V, true>(p, L.nch_f, s);
    return fwd_chain_rn<T, V, false>(p, L.nch_f, s);
}

hipError_t launch_fwd_chain(const rorbk_handle_s *h, const FwdArgs &a, const void *r,
                            double *ckst, hipStream_t s) {
    if (a.vec == VEC_F64) return fwd_chain_typed<double, double>(h, a, r, ckst, s);
    if (a.dt == RORBK_F32) return fwd_chain_typed<float, float>(h, a, r, ckst, s);
    return fwd_chain_typed<bf16_t, float>(h, a, r, ckst, s);
}

template <typename T>
static hipError_t gram_chain_typed(const rorbk_handle_s *h, const GramChainP &p, int aligned,
                                   hipStream_t s) {
    const int jobs = gram_chain_tiles(p.K, p.bmax) * h->L.nch_c;
    if (aligned)
        hipLaunchKernelGGL((k_gram_chain<T, true>), dim3(jobs), dim3(64 * GC_W), 0, s, p);
    else
        hipLaunchKernelGGL((k_gram_chain<T, false>), dim3(jobs), dim3(64 * GC_W), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_gram_chain(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                             const int32_t *I, int64_t ti, double *G, hipStream_t s) {
    const Layout &L = h->L;
    if (L.K > 64 || L.bmax > FWD_B || !h->d_C) return hipErrorInvalidValue;
    GramChainP p;
    p.A = A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.bmax = (int)L.bmax;
    p.I = I;
    p.K = (int)L.K;
    p.tau = h->d_tau;
    p.ti = ti;
    p.wc = L.wc;
    p.G = G;
    p.C = h->d_C;
    p.ctrl = h->d_ctrl;
    if (dt == RORBK_F64) return gram_chain_typed<double>(h, p, aligned, s);
    if (dt == RORBK_F32) return gram_chain_typed<float>(h, p, aligned, s);
    return gram_chain_typed<bf16_t>(h, p, aligned, s);
}

}  // namespace rorbk
