// k_csr.hip -- ROR-BK kernels for a CSR matrix (FP64 or FP32 values, int32
// column indices ascending within each row, int64 row offsets): input check,
// the residual SpMV, the block step, the greedy block's Gram, and the setup
// (centroids for the cosine proposal, fixed-block Grams by sparse row merges).
//
// A block of a sparse matrix holds a few thousand entries, so a block step is
// one workgroup: it stages the block's entries in LDS, forms the update, and
// adds it into x once per distinct column, in a fixed order (no floating-point
// atomics).  The residual pass is a plain SpMV over all rows.
#include "rorbk_device.h"

namespace rorbk {

// ------------------------------------------------------------ input check --
// rowptr[0] == 0, rowptr[m] == nnz, non-decreasing offsets, and column indices
// in [0, n) strictly ascending within each row; any violation sets *bad.
__global__ __launch_bounds__(256) void k_csr_check(const int64_t *__restrict__ rowptr,
                                                   const int32_t *__restrict__ colidx, int64_t m,
                                                   int64_t n, int64_t nnz, int32_t *__restrict__ bad) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i == 0 && (rowptr[0] != 0 || rowptr[m] != nnz)) *bad = 1;
    if (i >= m) return;
    const int64_t p0 = rowptr[i], p1 = rowptr[i + 1];
    if (p1 < p0 || p0 < 0 || p1 > nnz) {
        *bad = 1;
        return;
    }
    int64_t prev = -1;
    for (int64_t p = p0; p < p1; ++p) {
        const int64_t c = colidx[p];
        if (c <= prev || c >= n) {
            *bad = 1;
            return;
        }
        prev = c;
    }
}

// ------------------------------------------------------------------ SpMV --
// Algorithm 1, r = b - A x: (A x)_i for every row, SPMV_LPR lanes per row
// (entries strided over the lanes, lane sums combined by a fixed butterfly),
// written to axp[i] for the selection kernel.
constexpr int SPMV_LPR = 4;

template <typename T, typename V>
__global__ __launch_bounds__(256) void k_csr_spmv(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const T *__restrict__ val, int64_t m,
                                                  const V *__restrict__ x, double *__restrict__ axp,
                                                  const Ctrl *__restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    const int64_t row = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / SPMV_LPR;
    const int sub = threadIdx.x % SPMV_LPR;
    V acc = (V)0;
    if (row < m) {
        const int64_t p1 = rowptr[row + 1];
        for (int64_t p = rowptr[row] + sub; p < p1; p += SPMV_LPR)
            acc = fmaT((V)val[p], x[colidx[p]], acc);
    }
    acc = group_sum(acc, SPMV_LPR);
    if (row < m && sub == 0) axp[row] = (double)acc;
}

// ------------------------------------------------------- staged row sets --
constexpr int CSR_STAGE = 4096;   // entries of a row set held in LDS

// Exclusive prefix sums of len[0..R) (R <= 3 * 64) into off[0..R], by wave 0.
__device__ __forceinline__ void wave0_exscan(const int64_t *len, int R, int64_t *off) {
    if (threadIdx.x < WAVE) {
        const int lane = threadIdx.x;
        int64_t carry = 0;
        for (int c0 = 0; c0 < R; c0 += WAVE) {
            const int64_t v = (c0 + lane < R) ? len[c0 + lane] : 0;
            int64_t inc = v;
            for (int o = 1; o < WAVE; o <<= 1) {
                const int64_t t = __shfl_up(inc, o, WAVE);
                if (lane >= o) inc += t;
            }
            if (c0 + lane < R) off[c0 + lane] = carry + inc - v;
            carry += __shfl(inc, WAVE - 1, WAVE);
        }
        if (lane == 0) off[R] = carry;
    }
}

// Row r (0 <= r < R) of the set holding entry e: the last r with off[r] <= e.
__device__ __forceinline__ int row_of_entry(const int64_t *off, int R, int64_t e) {
    int lo = 0, hi = R;   // off[lo] <= e < off[hi]
    while (hi - lo > 1) {
        const int mid = (lo + hi) >> 1;
        if (off[mid] <= e) lo = mid;
        else hi = mid;
    }
    return lo;
}

// Sparse dot of two rows with ascending columns: the common columns in
// ascending order, summed sequentially.
template <typename VA>
__device__ __forceinline__ double merge_dot(const int32_t *ca, const VA *va, int64_t la,
                                            const int32_t *cb, const VA *vb, int64_t lb) {
    double s = 0.0;
    int64_t i = 0, j = 0;
    while (i < la && j < lb) {
        const int32_t a = ca[i], b = cb[j];
        if (a < b) ++i;
        else if (a > b) ++j;
        else {
            s = s + (double)va[i] * (double)vb[j];
            ++i;
            ++j;
        }
    }
    return s;
}

// (i, j), j <= i, of packed lower index f = i (i + 1) / 2 + j.
__device__ __forceinline__ void unpack_lower(int64_t f, int *i, int *j) {
    int a = (int)((sqrt(8.0 * (double)f + 1.0) - 1.0) * 0.5);
    while ((int64_t)(a + 1) * (a + 2) / 2 <= f) ++a;
    while ((int64_t)a * (a + 1) / 2 > f) --a;
    *i = a;
    *j = (int)(f - (int64_t)a * (a + 1) / 2);
}

// Lower triangle of the Gram of R sparse rows (row r = rows[r], or first + r
// when rows == NULL): packed G[pk(i, j)] = <A_(i), A_(j)>, one entry per
// thread over [f0, f1).  The rows are staged in LDS when they fit.
template <typename T>
__device__ void sparse_gram(const int64_t *__restrict__ rowptr, const int32_t *__restrict__ colidx,
                            const T *__restrict__ val, const int32_t *__restrict__ rows,
                            int64_t first, int R, int64_t f0, int64_t f1, double *__restrict__ G) {
    __shared__ int32_t s_c[CSR_STAGE];
    __shared__ double s_v[CSR_STAGE];
    __shared__ int64_t s_len[MAXB], s_off[MAXB + 1], s_p0[MAXB];
    for (int r = threadIdx.x; r < R; r += blockDim.x) {
        const int64_t row = rows ? (int64_t)rows[r] : first + r;
        const int64_t p0 = rowptr[row];
        s_p0[r] = p0;
        s_len[r] = rowptr[row + 1] - p0;
    }
    __syncthreads();
    wave0_exscan(s_len, R, s_off);
    __syncthreads();
    const int64_t tot = s_off[R];
    const bool staged = tot <= CSR_STAGE;
    if (staged) {
        for (int64_t e = threadIdx.x; e < tot; e += blockDim.x) {
            const int r = row_of_entry(s_off, R, e);
            const int64_t p = s_p0[r] + (e - s_off[r]);
            s_c[e] = colidx[p];
            s_v[e] = (double)val[p];
        }
    }
    __syncthreads();
    for (int64_t f = f0 + threadIdx.x; f < f1; f += blockDim.x) {
        int i, j;
        unpack_lower(f, &i, &j);
        double s;
        if (staged)
            s = merge_dot<double>(s_c + s_off[i], s_v + s_off[i], s_len[i], s_c + s_off[j],
                                  s_v + s_off[j], s_len[j]);
        else
            s = merge_dot<T>(colidx + s_p0[i], val + s_p0[i], s_len[i], colidx + s_p0[j],
                             val + s_p0[j], s_len[j]);
        G[f] = s;
    }
}

// Fixed-block Grams for the stored inverses (Section 3.1): one workgroup per
// block, packed lower output Gs[t][pk(i,j)].
template <typename T>
__global__ __launch_bounds__(256) void k_csr_block_gram(const int64_t *__restrict__ rowptr,
                                                        const int32_t *__restrict__ colidx,
                                                        const T *__restrict__ val, int64_t q,
                                                        int64_t rem, int64_t kpmax,
                                                        double *__restrict__ Gs) {
    const int64_t t = blockIdx.x;
    const int bt = blk_rows(t, q, rem);
    sparse_gram<T>(rowptr, colidx, val, nullptr, blk_start(t, q, rem), bt, 0,
                   (int64_t)bt * (bt + 1) / 2, Gs + t * kpmax);
}

// The greedy block's Gram A_I A_I^T (Algorithm 1): workgroup w computes packed
// entries [256 w, 256 (w + 1)); output is chunk 0 of the Gram partials.
template <typename T>
__global__ __launch_bounds__(256) void k_csr_gram(const int64_t *__restrict__ rowptr,
                                                  const int32_t *__restrict__ colidx,
                                                  const T *__restrict__ val,
                                                  const int32_t *__restrict__ idx, int K,
                                                  double *__restrict__ G,
                                                  const Ctrl *__restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    const int64_t KP = (int64_t)K * (K + 1) / 2;
    const int64_t f0 = (int64_t)blockIdx.x * 256;
    const int64_t f1 = (f0 + 256 < KP) ? f0 + 256 : KP;
    sparse_gram<T>(rowptr, colidx, val, idx, 0, K, f0, f1, G);
}

// Centroids for the cosine proposal (Algorithm 1, first step): cen[t][col] is
// the sum of block t's rows, added in ascending row order (one row at a time;
// a row's columns are distinct, so its entries go in parallel).
template <typename T>
__global__ __launch_bounds__(256) void k_csr_centroid(const int64_t *__restrict__ rowptr,
                                                      const int32_t *__restrict__ colidx,
                                                      const T *__restrict__ val, int64_t n,
                                                      int64_t q, int64_t rem,
                                                      double *__restrict__ cen) {
    const int64_t t = blockIdx.x;
    const int64_t r0 = blk_start(t, q, rem);
    const int bt = blk_rows(t, q, rem);
    double *c = cen + t * n;
    for (int r = 0; r < bt; ++r) {
        const int64_t p1 = rowptr[r0 + r + 1];
        for (int64_t p = rowptr[r0 + r] + threadIdx.x; p < p1; p += blockDim.x)
            c[colidx[p]] += (double)val[p];
        __syncthreads();
    }
}

// ------------------------------------------------------------ block step --
// One regularised block update of Lemma 2 / Algorithm 1 on a sparse block,
// fused with the next step's products, in one workgroup:
//   1. (ymode 0) r_S = b_S - Pin (A_S x from the previous kernel), y = H_t r_S
//      with the stored inverse of block t; (ymode 1) y given; (ymode 2) no
//      update;
//   2. x += A_S^T y: the block's entries are taken in row order, in chunks of
//      CSR_CHUNK; within a chunk each entry's column goes to a hash slot; a
//      column with one term a_ij y_i gets x_j + term, a column with several
//      gets x_j + (their sum in row order), so every x_j is written once per
//      chunk by one thread;
//   3. Pout[i] = A_{S'} x for the next step's rows S' (entry products summed in
//      entry order per row).
// Everything that does not depend on y or on the new x is fetched first: the
// row offsets, the first chunk's entries and their hash slots, and the next
// rows' entries (when they fit CSR_NCAP), so the dependent part is the stored
// inverse product, one read-modify-write of x and one gather of x.
// With b == NULL the step is the adjoint one: gb[S] -= y.
constexpr int CSR_STEP_T = 512;
constexpr int CSR_CHUNK = 2048;         // entries per update chunk
constexpr int CSR_HASH = 4096;          // hash slots (a power of two >= 2 * CSR_CHUNK)
constexpr int CSR_HASH_BITS = 12;
constexpr int CSR_NCAP = 2048;          // next-row entries prefetched (4 per thread)
constexpr int CSR_TPR = 4;              // threads per row of the stored-inverse product

struct CsrStepP {
    const int64_t *rowptr;
    const int32_t *colidx;
    const void *val;
    int64_t m, n, q, rem;
    const int32_t *tau;
    RowSel cur;
    int ymode;
    const double *Pin;
    const double *H;
    const void *b;
    void *x;
    void *gb;
    const double *ygiven;
    RowSel nxt;
    double *Pout;
    const Ctrl *ctrl;
};

// Entries [base, base + ne) of the row set (offsets off, starts p0) into the
// chunk arrays: column, value, local row, and a hash slot per distinct column
// (h_cnt: entries per slot, h_head: the first entry of the slot).
template <typename T, typename V>
__device__ __forceinline__ void csr_stage_chunk(const int32_t *__restrict__ colidx,
                                                const T *__restrict__ val, const int64_t *off,
                                                const int64_t *p0, int cnt, int64_t base, int ne,
                                                int32_t *e_col, V *e_val, int16_t *e_row,
                                                int32_t *e_slot, int32_t *h_key, int32_t *h_head,
                                                uint32_t *h_cnt) {
    for (int e = threadIdx.x; e < ne; e += CSR_STEP_T) {
        const int64_t ge = base + e;
        const int r = row_of_entry(off, cnt, ge);
        const int64_t pp = p0[r] + (ge - off[r]);
        const int32_t c = colidx[pp];
        e_col[e] = c;
        e_val[e] = (V)val[pp];
        e_row[e] = (int16_t)r;
        uint32_t sl = ((uint32_t)c * 2654435761u) >> (32 - CSR_HASH_BITS);
        while (true) {
            const int32_t old = atomicCAS(&h_key[sl], -1, c);
            if (old == -1 || old == c) break;
            sl = (sl + 1) & (CSR_HASH - 1);
        }
        e_slot[e] = (int32_t)sl;
        atomicAdd(&h_cnt[sl], 1u);
        atomicMin(&h_head[sl], e);
    }
}

__device__ __forceinline__ void csr_clear_hash(int32_t *h_key, int32_t *h_head, uint32_t *h_cnt) {
    for (int s = threadIdx.x; s < CSR_HASH; s += CSR_STEP_T) {
        h_key[s] = -1;
        h_head[s] = 0x7fffffff;
        h_cnt[s] = 0u;
    }
}

// x += the staged chunk's terms e_val[e] * y[e_row[e]]: one write per column.
template <typename V>
__device__ __forceinline__ void csr_apply_chunk(V *__restrict__ x, int ne, const double *s_y,
                                                const int32_t *e_col, V *e_val,
                                                const int16_t *e_row, const int32_t *e_slot,
                                                const int32_t *h_head, const uint32_t *h_cnt,
                                                int32_t *s_dup, int *s_ndup) {
    const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
    constexpr int NW = CSR_STEP_T / WAVE;
    for (int e = tid; e < ne; e += CSR_STEP_T) e_val[e] = e_val[e] * (V)s_y[e_row[e]];
    __syncthreads();
    for (int e = tid; e < ne; e += CSR_STEP_T) {
        const int sl = e_slot[e];
        if (h_head[sl] == e) {
            if (h_cnt[sl] == 1u) {
                const int32_t c = e_col[e];
                x[c] = x[c] + e_val[e];
            } else {
                s_dup[atomicAdd(s_ndup, 1)] = e;
            }
        }
    }
    __syncthreads();
    // columns with several terms: one wave each, terms in entry order
    const int nd = *s_ndup;
    for (int d = wv; d < nd; d += NW) {
        const int e0 = s_dup[d];
        const int sl = e_slot[e0];
        V acc = (V)0;
        for (int b0 = e0; b0 < ne; b0 += WAVE) {
            const int e = b0 + lane;
            const bool hit = e < ne && e_slot[e] == sl;
            unsigned long long bits = __ballot(hit);
            if (lane == 0) {
                while (bits) {
                    const int bit = __ffsll((long long)bits) - 1;
                    acc = acc + e_val[b0 + bit];
                    bits &= bits - 1;
                }
            }
        }
        if (lane == 0) {
            const int32_t c = e_col[e0];
            x[c] = x[c] + acc;
        }
    }
    __syncthreads();
}

template <typename T, typename V>
__global__ __launch_bounds__(CSR_STEP_T) void k_csr_step(CsrStepP p) {
    const int tid = threadIdx.x;
    const T *__restrict__ val = (const T *)p.val;
    V *__restrict__ x = (V *)p.x;
    const V *__restrict__ b = (const V *)p.b;
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
    const bool upd = p.ymode != 2 && cnt > 0;

    __shared__ double s_r[MAXB], s_y[MAXB];
    __shared__ int64_t s_len[MAXB], s_off[MAXB + 1], s_p0[MAXB];
    __shared__ int64_t n_len[MAXB], n_off[MAXB + 1], n_p0[MAXB];
    __shared__ int32_t e_col[CSR_CHUNK], e_slot[CSR_CHUNK], s_dup[CSR_CHUNK];
    __shared__ int16_t e_row[CSR_CHUNK];
    __shared__ V e_val[CSR_CHUNK];
    __shared__ V n_prod[CSR_NCAP];
    __shared__ int32_t h_key[CSR_HASH], h_head[CSR_HASH];
    __shared__ uint32_t h_cnt[CSR_HASH];
    __shared__ int s_ndup;

    // A. row offsets of both row sets; b - Pin or the given y
    if (upd) {
        for (int i = tid; i < cnt; i += CSR_STEP_T) {
            const int64_t row = (p.cur.kind == 1) ? (int64_t)p.cur.idx[i] : cst + i;
            const int64_t p0 = p.rowptr[row];
            s_p0[i] = p0;
            s_len[i] = p.rowptr[row + 1] - p0;
            if (p.ymode == 0) s_r[i] = (b ? (double)b[row] : 0.0) - p.Pin[i];
            else s_y[i] = p.ygiven[i];
        }
    }
    for (int i = tid; i < ncnt; i += CSR_STEP_T) {
        const int64_t row = (p.nxt.kind == 1) ? (int64_t)p.nxt.idx[i] : nst + i;
        const int64_t p0 = p.rowptr[row];
        n_p0[i] = p0;
        n_len[i] = p.rowptr[row + 1] - p0;
    }
    if (upd) csr_clear_hash(h_key, h_head, h_cnt);
    if (tid == 0) s_ndup = 0;
    __syncthreads();
    if (upd) wave0_exscan(s_len, cnt, s_off);
    if (ncnt > 0 && tid >= WAVE && tid < 2 * WAVE) {
        // the same scan on wave 1 for the next rows
        const int lane = tid - WAVE;
        int64_t carry = 0;
        for (int c0 = 0; c0 < ncnt; c0 += WAVE) {
            const int64_t v = (c0 + lane < ncnt) ? n_len[c0 + lane] : 0;
            int64_t inc = v;
            for (int o = 1; o < WAVE; o <<= 1) {
                const int64_t t = __shfl_up(inc, o, WAVE);
                if (lane >= o) inc += t;
            }
            if (c0 + lane < ncnt) n_off[c0 + lane] = carry + inc - v;
            carry += __shfl(inc, WAVE - 1, WAVE);
        }
        if (lane == 0) n_off[ncnt] = carry;
    }
    __syncthreads();
    const int64_t tot = upd ? s_off[cnt] : 0;
    const int64_t ntot = (ncnt > 0) ? n_off[ncnt] : 0;
    // B. the next rows' entries (x-independent) into registers
    const bool npre = ntot <= CSR_NCAP;
    constexpr int NU = CSR_NCAP / CSR_STEP_T;
    int32_t ncol[NU];
    T nval[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int e = tid + u * CSR_STEP_T;
        ncol[u] = 0;
        nval[u] = (T)0;
        if (npre && e < ntot) {
            const int r = row_of_entry(n_off, ncnt, e);
            const int64_t pp = n_p0[r] + (e - n_off[r]);
            ncol[u] = p.colidx[pp];
            nval[u] = val[pp];
        }
    }
    // C. the first chunk of this block's entries with their hash slots
    const int ne0 = (int)((tot < CSR_CHUNK) ? tot : CSR_CHUNK);
    if (upd)
        csr_stage_chunk<T, V>(p.colidx, val, s_off, s_p0, cnt, 0, ne0, e_col, e_val, e_row,
                              e_slot, h_key, h_head, h_cnt);
    // D. y = H_t r_S: CSR_TPR threads per row, rows i0 and i0 + 128 per thread,
    //    every load of both rows in flight at once
    if (upd && p.ymode == 0) {
        const double *__restrict__ H = p.H + blk_hoff(tc, p.q, p.rem);
        constexpr int HU = (MAXB + CSR_TPR - 1) / CSR_TPR;
        constexpr int RPP = CSR_STEP_T / CSR_TPR;   // rows per pass (MAXB <= 2 * RPP)
        static_assert(MAXB <= 2 * RPP, "two row slots per thread cover a block");
        const int qd = tid % CSR_TPR, i0 = tid / CSR_TPR, i1 = i0 + RPP;
        double h0[HU], h1[HU];
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            const int j = qd + CSR_TPR * u;
            h0[u] = (i0 < cnt && j < cnt) ? H[(int64_t)j * cnt + i0] : 0.0;
            h1[u] = (i1 < cnt && j < cnt) ? H[(int64_t)j * cnt + i1] : 0.0;
        }
        double s0 = 0.0, s1 = 0.0;
#pragma unroll
        for (int u = 0; u < HU; ++u) {
            const int j = qd + CSR_TPR * u;
            if (j < cnt) {
                s0 = __builtin_fma(h0[u], s_r[j], s0);
                s1 = __builtin_fma(h1[u], s_r[j], s1);
            }
        }
        s0 = group_sum(s0, CSR_TPR);
        s1 = group_sum(s1, CSR_TPR);
        if (qd == 0) {
            if (i0 < cnt) s_y[i0] = s0;
            if (i1 < cnt) s_y[i1] = s1;
        }
    }
    __syncthreads();
    if (upd && p.gb) {
        V *gb = (V *)p.gb;
        for (int i = tid; i < cnt; i += CSR_STEP_T) {
            const int64_t row = (p.cur.kind == 1) ? (int64_t)p.cur.idx[i] : cst + i;
            gb[row] -= (V)s_y[i];
        }
    }
    // E. x += A_S^T y, chunk by chunk
    if (upd) {
        csr_apply_chunk<V>(x, ne0, s_y, e_col, e_val, e_row, e_slot, h_head, h_cnt, s_dup,
                           &s_ndup);
        for (int64_t base = CSR_CHUNK; base < tot; base += CSR_CHUNK) {
            const int ne = (int)((tot - base < CSR_CHUNK) ? tot - base : CSR_CHUNK);
            csr_clear_hash(h_key, h_head, h_cnt);
            if (tid == 0) s_ndup = 0;
            __syncthreads();
            csr_stage_chunk<T, V>(p.colidx, val, s_off, s_p0, cnt, base, ne, e_col, e_val, e_row,
                                  e_slot, h_key, h_head, h_cnt);
            __syncthreads();
            csr_apply_chunk<V>(x, ne, s_y, e_col, e_val, e_row, e_slot, h_head, h_cnt, s_dup,
                               &s_ndup);
        }
    }
    // F. products of the next rows with the updated x
    if (ncnt > 0) {
        if (npre) {
#pragma unroll
            for (int u = 0; u < NU; ++u) {
                const int e = tid + u * CSR_STEP_T;
                if (e < ntot) n_prod[e] = (V)nval[u] * x[ncol[u]];
            }
            __syncthreads();
            for (int i = tid; i < ncnt; i += CSR_STEP_T) {
                V acc = (V)0;
                const int e1 = (int)n_off[i + 1];
                for (int e = (int)n_off[i]; e < e1; ++e) acc = acc + n_prod[e];
                p.Pout[i] = (double)acc;
            }
        } else {
            const int sub = tid % SPMV_LPR;
            for (int i0 = 0; i0 < ncnt; i0 += CSR_STEP_T / SPMV_LPR) {
                const int i = i0 + tid / SPMV_LPR;
                V acc = (V)0;
                if (i < ncnt) {
                    const int64_t e1 = n_p0[i] + n_len[i];
                    for (int64_t pp = n_p0[i] + sub; pp < e1; pp += SPMV_LPR)
                        acc = fmaT((V)val[pp], x[p.colidx[pp]], acc);
                }
                acc = group_sum(acc, SPMV_LPR);
                if (i < ncnt && sub == 0) p.Pout[i] = (double)acc;
            }
        }
    }
}

// ------------------------------------------------------------ launchers --
hipError_t launch_csr_check(const rorbk_handle_s *h, int32_t *bad, hipStream_t s) {
    const Layout &L = h->L;
    hipLaunchKernelGGL(k_csr_check, dim3((unsigned)((L.m + 255) / 256)), dim3(256), 0, s,
                       h->rowptr, h->colidx, L.m, L.n, L.nnz, bad);
    return hipGetLastError();
}

hipError_t launch_residual_csr(const rorbk_handle_s *h, const void *vals, int dt, int vec,
                               const void *x, double *axp, hipStream_t s) {
    const Layout &L = h->L;
    const unsigned grid = (unsigned)((L.m * SPMV_LPR + 255) / 256);
    if (vec == VEC_F64) {
        if (dt != RORBK_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_csr_spmv<double, double>), dim3(grid), dim3(256), 0, s, h->rowptr,
                           h->colidx, (const double *)vals, L.m, (const double *)x, axp,
                           (const Ctrl *)h->d_ctrl);
    } else {
        if (dt != RORBK_F32) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_csr_spmv<float, float>), dim3(grid), dim3(256), 0, s, h->rowptr,
                           h->colidx, (const float *)vals, L.m, (const float *)x, axp,
                           (const Ctrl *)h->d_ctrl);
    }
    return hipGetLastError();
}

hipError_t launch_step_csr(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    CsrStepP p;
    p.rowptr = h->rowptr;
    p.colidx = h->colidx;
    p.val = a.A;
    p.m = L.m;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.tau = h->d_tau;
    p.cur = a.cur;
    p.ymode = a.ymode;
    p.Pin = a.Pin;
    p.H = h->d_H;
    p.b = a.b;
    p.x = a.x;
    p.gb = a.gb;
    p.ygiven = a.ygiven;
    p.nxt = a.nxt;
    p.Pout = a.Pout;
    p.ctrl = h->d_ctrl;
    if (a.vec == VEC_F64) {
        if (a.dt != RORBK_F64) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_csr_step<double, double>), dim3(1), dim3(CSR_STEP_T), 0, s, p);
    } else {
        if (a.dt != RORBK_F32) return hipErrorInvalidValue;
        hipLaunchKernelGGL((k_csr_step<float, float>), dim3(1), dim3(CSR_STEP_T), 0, s, p);
    }
    return hipGetLastError();
}

hipError_t launch_gram_csr(const rorbk_handle_s *h, const void *vals, int dt, const int32_t *idx,
                           int K, double *G, hipStream_t s) {
    const int64_t KP = (int64_t)K * (K + 1) / 2;
    const unsigned grid = (unsigned)((KP + 255) / 256);
    if (dt == RORBK_F64)
        hipLaunchKernelGGL(k_csr_gram<double>, dim3(grid), dim3(256), 0, s, h->rowptr, h->colidx,
                           (const double *)vals, idx, K, G, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL(k_csr_gram<float>, dim3(grid), dim3(256), 0, s, h->rowptr, h->colidx,
                           (const float *)vals, idx, K, G, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_setup_proposal_csr(const rorbk_handle_s *h, const void *vals, int dt,
                                     double *scratch, hipStream_t s) {
    const Layout &L = h->L;
    double *cen = scratch;                      // k * n
    double *nrm = cen + L.k * L.n;              // k
    double *Sp = nrm + L.k;                     // k * ntc
    hipError_t e = launch_fill_zero(cen, (int64_t)sizeof(double) * L.k * L.n, s);
    if (e != hipSuccess) return e;
    if (dt == RORBK_F64)
        hipLaunchKernelGGL(k_csr_centroid<double>, dim3((unsigned)L.k), dim3(256), 0, s, h->rowptr,
                           h->colidx, (const double *)vals, L.n, L.q, L.rem, cen);
    else
        hipLaunchKernelGGL(k_csr_centroid<float>, dim3((unsigned)L.k), dim3(256), 0, s, h->rowptr,
                           h->colidx, (const float *)vals, L.n, L.q, L.rem, cen);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_colsum(cen, L.k, L.n, h->d_ysum, s);     // the row sum of A (Algorithm 2)
    if (e != hipSuccess) return e;
    return launch_proposal_from_centroids(h, cen, nrm, Sp, s);
}

hipError_t launch_block_inverses_csr(const rorbk_handle_s *h, const void *vals, int dt,
                                     int32_t *d_fail, hipStream_t s) {
    const Layout &L = h->L;
    const int64_t kp = L.bmax * (L.bmax + 1) / 2;
    double *Gs = nullptr;
    hipError_t e = hipMallocAsync((void **)&Gs, sizeof(double) * (size_t)(kp * L.k), s);
    if (e != hipSuccess) return e;
    if (dt == RORBK_F64)
        hipLaunchKernelGGL(k_csr_block_gram<double>, dim3((unsigned)L.k), dim3(256), 0, s,
                           h->rowptr, h->colidx, (const double *)vals, L.q, L.rem, kp, Gs);
    else
        hipLaunchKernelGGL(k_csr_block_gram<float>, dim3((unsigned)L.k), dim3(256), 0, s,
                           h->rowptr, h->colidx, (const float *)vals, L.q, L.rem, kp, Gs);
    e = hipGetLastError();
    if (e == hipSuccess) e = launch_block_inverses_from_grams(h, Gs, kp, d_fail, s);
    hipError_t e2 = hipFreeAsync(Gs, s);
    return e != hipSuccess ? e : e2;
}

}  // namespace rorbk
