// k_dense.hip -- ROR-BK kernels for a dense row-major matrix (FP64, FP32 or
// BF16 storage): the full residual pass, the fused block step, the greedy
// block's Gram, and the setup (centroid cosines, proposal, block inverses).
#include "rorbk_device.h"

namespace rorbk {

constexpr int SEG = 2048;  // columns of one residual segment (x kept in VGPRs)

// ------------------------------------------------------------ residual pass --
// Algorithm 1, r = b - A x: the products (A x)_i over one 2048-column segment.
// One wave per row, each lane holding its 32 entries of x in registers and
// streaming the row with 16-byte non-temporal loads; the lane sums are combined
// by a fixed butterfly.  axp[seg][i] = partial (A x)_i; the selection kernel
// subtracts the segment sum from b.  Grid: x = row groups (4 waves of `rpw`
// rows), y = segments.
template <typename T, typename V, bool AL>
__global__ __launch_bounds__(256) void k_resid_dense(const T *__restrict__ A, int64_t ld,
                                                     int64_t m, int64_t n,
                                                     const V *__restrict__ x,
                                                     double *__restrict__ axp, int rpw,
                                                     const Ctrl *__restrict__ ctrl) {
    if (ctrl && ctrl->done) return;
    constexpr int VW = Tr<T>::VW;
    constexpr int NVL = SEG / (WAVE * VW);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t seg = blockIdx.y;
    const int64_t c0 = seg * SEG;
    V xr[NVL][VW];
#pragma unroll
    for (int s = 0; s < NVL; ++s) {
        const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW;
#pragma unroll
        for (int e = 0; e < VW; ++e) xr[s][e] = (col + e < n) ? x[col + e] : (V)0;
    }
    const int64_t r0 = ((int64_t)blockIdx.x * 4 + w) * rpw;
    for (int rr = 0; rr < rpw; ++rr) {
        const int64_t i = r0 + rr;
        if (i >= m) break;
        const T *row = A + i * ld;
        V acc = (V)0;
#pragma unroll
        for (int s = 0; s < NVL; ++s) {
            const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW;
            if (col < n) {
                V a[VW];
                load_vec_nt<T, V, AL>(row, col, n, a);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc = fmaT(a[e], xr[s][e], acc);
            }
        }
        acc = group_sum(acc, WAVE);
        if (lane == 0) axp[seg * m + i] = (double)acc;
    }
}

// ------------------------------------------------------------ block step --
// One regularised block update (Lemma 2's update rule, Algorithm 1) fused with
// the partial products of the next step.  Workgroup w owns columns
// [w*wu, (w+1)*wu):
//   1. (ymode 0) r_S = b_S - sum_ch Pin[ch][.] (chunk order), y = H_t r_S with
//      the stored inverse H_t of block t; (ymode 1) y given;
//   2. x[cols] += A_S[:, cols]^T y (rows split over row groups, summed in
//      group order);
//   3. Pout[w][p] = A_{S'}[p, cols] . x[cols] for the next step's rows S'.
// With b == NULL the step is the adjoint one (see the backward pass): then
// workgroup 0 also accumulates gb[S] -= y.
struct StepP {
    const void *A;
    int64_t ld, m, n;
    const int64_t *off;
    const int32_t *tau;
    RowSel cur;
    int ymode;
    const double *Pin;
    int nch;
    int bmax;
    const double *H;
    const int64_t *hoff;
    const void *b;
    void *x;
    void *gb;
    const double *ygiven;
    RowSel nxt;
    double *Pout;
    int64_t wu;
    const Ctrl *ctrl;
};

template <typename V>
__device__ __forceinline__ void resolve_rows(const RowSel &s, const int64_t *off, const int32_t *tau,
                                             int64_t *start, int *cnt, int *t) {
    if (s.kind == 0) {
        *t = tau[s.tau_index];
        *start = off[*t];
        *cnt = (int)(off[*t + 1] - *start);
    } else if (s.kind == 1) {
        *t = -1;
        *start = 0;
        *cnt = s.count;
    } else {
        *t = -1;
        *start = 0;
        *cnt = 0;
    }
}

template <typename T, typename V, bool AL>
__global__ __launch_bounds__(256) void k_step_dense(StepP p) {
    if (p.ctrl->done) return;
    constexpr int VW = Tr<T>::VW;
    constexpr int NV = 128 / VW;   // threads across a 128-column slab
    constexpr int G = 256 / NV;    // row groups
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const V *__restrict__ b = (const V *)p.b;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;
    const int64_t c0 = (int64_t)blockIdx.x * p.wu;
    const int64_t c1 = (c0 + p.wu < p.n) ? c0 + p.wu : p.n;
    const int wcols = (int)(c1 - c0);
    __shared__ V s_x[1024];
    __shared__ V s_red[G][128];
    __shared__ double s_r[MAXB], s_y[MAXB];
    __shared__ int64_t s_row[MAXB];

    int64_t start;
    int cnt, t;
    resolve_rows<V>(p.cur, p.off, p.tau, &start, &cnt, &t);
    for (int i = tid; i < cnt; i += 256)
        s_row[i] = (p.cur.kind == 1) ? (int64_t)p.cur.idx[i] : start + i;
    for (int c = tid; c < wcols; c += 256) s_x[c] = x[c0 + c];
    __syncthreads();

    if (p.ymode == 0) {
        for (int i = tid; i < cnt; i += 256) {
            double s = 0.0;
            for (int ch = 0; ch < p.nch; ++ch) s += p.Pin[(int64_t)ch * p.bmax + i];
            const double bi = b ? (double)b[s_row[i]] : 0.0;
            s_r[i] = bi - s;
        }
        __syncthreads();
        const double *__restrict__ H = p.H + p.hoff[t];
        for (int i = tid; i < cnt; i += 256) {
            double y = 0.0;
            for (int j = 0; j < cnt; ++j) y = __builtin_fma(H[(int64_t)j * cnt + i], s_r[j], y);
            s_y[i] = y;
        }
        __syncthreads();
    } else if (p.ymode == 1) {
        for (int i = tid; i < cnt; i += 256) s_y[i] = p.ygiven[i];
        __syncthreads();
    }
    if (p.gb && p.ymode != 2 && blockIdx.x == 0) {
        V *gb = (V *)p.gb;
        for (int i = tid; i < cnt; i += 256) gb[s_row[i]] -= (V)s_y[i];
    }

    if (p.ymode != 2) {
        for (int64_t sub = c0; sub < c1; sub += 128) {
            V acc[VW];
#pragma unroll
            for (int e = 0; e < VW; ++e) acc[e] = (V)0;
            const int64_t col = sub + (int64_t)v * VW;
            if (col < c1) {
                for (int q = g; q < cnt; q += G) {
                    V a[VW];
                    load_vec<T, V, AL>(A + s_row[q] * p.ld, col, c1, a);
                    const V yv = (V)s_y[q];
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[e] = fmaT(a[e], yv, acc[e]);
                }
            }
#pragma unroll
            for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
            __syncthreads();
            if (tid < 128) {
                const int64_t cc = sub + tid;
                if (cc < c1) {
                    V s = (V)0;
                    for (int gg = 0; gg < G; ++gg) s += s_red[gg][tid];
                    s_x[cc - c0] += s;
                }
            }
            __syncthreads();
        }
        for (int c = tid; c < wcols; c += 256) x[c0 + c] = s_x[c];
    }

    if (p.nxt.kind >= 0) {
        int64_t nstart;
        int ncnt, nt;
        resolve_rows<V>(p.nxt, p.off, p.tau, &nstart, &ncnt, &nt);
        for (int q = g; q < ncnt; q += G) {
            const int64_t row = (p.nxt.kind == 1) ? (int64_t)p.nxt.idx[q] : nstart + q;
            const T *ar = A + row * p.ld;
            V acc = (V)0;
            for (int64_t sub = c0; sub < c1; sub += 128) {
                const int64_t col = sub + (int64_t)v * VW;
                if (col < c1) {
                    V a[VW];
                    load_vec<T, V, AL>(ar, col, c1, a);
#pragma unroll
                    for (int e = 0; e < VW; ++e)
                        if (col + e < c1) acc = fmaT(a[e], s_x[col + e - c0], acc);
                }
            }
            acc = group_sum(acc, NV);
            if (v == 0) p.Pout[(int64_t)blockIdx.x * p.bmax + q] = (double)acc;
        }
    }
}

// ------------------------------------------------------------ block Gram --
// Lower triangle of A_S A_S^T over a column range, accumulated in FP64 (the
// block Gram of the greedy step, Algorithm 1).  A 32-column tile of the rows
// is staged in LDS transposed ([column][row]); thread t owns one MT x MT
// micro-tile of the lower triangle of tiles.
constexpr int GT = 32;  // columns per LDS tile

template <typename T, int MT>
__device__ __forceinline__ void gram_accumulate(const T *__restrict__ A, int64_t ld,
                                                const int64_t *rows, int K, int64_t c0,
                                                int64_t c1, double (&acc)[MT][MT], int bi,
                                                int bj, double (*At)[MAXB + 8]) {
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int w = 0; w < MT; ++w) acc[u][w] = 0.0;
    for (int64_t cb = c0; cb < c1; cb += GT) {
        const int tc = (int)((cb + GT < c1) ? GT : (c1 - cb));
        for (int e = threadIdx.x; e < K * GT; e += blockDim.x) {
            const int q = e / GT, c = e % GT;
            At[c][q] = (c < tc) ? (double)to_v<double>(A[rows[q] * ld + cb + c]) : 0.0;
        }
        __syncthreads();
        if (bi >= 0) {
            for (int c = 0; c < tc; ++c) {
                double a[MT], bb[MT];
#pragma unroll
                for (int u = 0; u < MT; ++u) {
                    a[u] = At[c][bi * MT + u];
                    bb[u] = At[c][bj * MT + u];
                }
#pragma unroll
                for (int u = 0; u < MT; ++u)
#pragma unroll
                    for (int w = 0; w < MT; ++w) acc[u][w] = __builtin_fma(a[u], bb[w], acc[u][w]);
            }
        }
        __syncthreads();
    }
}

__device__ __forceinline__ void tile_of(int t, int nt, int *bi, int *bj) {
    // t-th tile of the lower triangle of an nt x nt tile grid, row-major
    int i = 0, base = 0;
    while (i < nt && base + i + 1 <= t) { base += i + 1; ++i; }
    if (i >= nt) { *bi = -1; *bj = -1; return; }
    *bi = i;
    *bj = t - base;
}

template <typename T, int MT>
__global__ __launch_bounds__(256) void k_gram_dense(const T *__restrict__ A, int64_t ld, int64_t n,
                                                    const int32_t *__restrict__ idx, int K,
                                                    int64_t wg, double *__restrict__ Gpart,
                                                    const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double At[GT][MAXB + 8];
    __shared__ int64_t rows[MAXB];
    for (int q = threadIdx.x; q < K; q += blockDim.x) rows[q] = idx[q];
    for (int e = threadIdx.x; e < GT * (MAXB + 8); e += blockDim.x) (&At[0][0])[e] = 0.0;
    __syncthreads();
    const int nt = (K + MT - 1) / MT;
    int bi = -1, bj = -1;
    if ((int)threadIdx.x < nt * (nt + 1) / 2) tile_of(threadIdx.x, nt, &bi, &bj);
    const int64_t c0 = (int64_t)blockIdx.x * wg;
    const int64_t c1 = (c0 + wg < n) ? c0 + wg : n;
    double acc[MT][MT];
    gram_accumulate<T, MT>(A, ld, rows, K, c0, c1, acc, bi, bj, At);
    if (bi >= 0) {
        double *Gp = Gpart + (int64_t)blockIdx.x * K * K;
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
            for (int w = 0; w < MT; ++w) {
                const int i = bi * MT + u, j = bj * MT + w;
                if (i < K && j <= i) Gp[i * K + j] = acc[u][w];
            }
    }
}

// ------------------------------------------------------------ launchers --
template <typename T, typename V>
static hipError_t step_typed(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    StepP p;
    p.A = a.A;
    p.ld = L.ld;
    p.m = L.m;
    p.n = L.n;
    p.off = h->d_off;
    p.tau = h->d_tau;
    p.cur = a.cur;
    p.ymode = a.ymode;
    p.Pin = a.Pin;
    p.nch = L.nch_u;
    p.bmax = (int)L.bmax;
    p.H = h->d_H;
    p.hoff = h->d_hoff;
    p.b = a.b;
    p.x = a.x;
    p.gb = a.gb;
    p.ygiven = a.ygiven;
    p.nxt = a.nxt;
    p.Pout = a.Pout;
    p.wu = L.wu;
    p.ctrl = h->d_ctrl;
    if (a.aligned)
        hipLaunchKernelGGL((k_step_dense<T, V, true>), dim3(L.nch_u), dim3(256), 0, s, p);
    else
        hipLaunchKernelGGL((k_step_dense<T, V, false>), dim3(L.nch_u), dim3(256), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_step_dense(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    if (a.vec == VEC_F64) return step_typed<double, double>(h, a, s);
    if (a.dt == RORBK_F32) return step_typed<float, float>(h, a, s);
    return step_typed<bf16_t, float>(h, a, s);
}

template <typename T, typename V>
static hipError_t resid_typed(const rorbk_handle_s *h, const void *A, int aligned,
                              const void *x, double *axp, hipStream_t s) {
    const Layout &L = h->L;
    const int rpw = 4;
    const int64_t groups = (L.m + 4 * rpw - 1) / (4 * rpw);
    dim3 grid((unsigned)groups, (unsigned)L.nseg);
    if (aligned)
        hipLaunchKernelGGL((k_resid_dense<T, V, true>), grid, dim3(256), 0, s, (const T *)A, L.ld,
                           L.m, L.n, (const V *)x, axp, rpw, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_resid_dense<T, V, false>), grid, dim3(256), 0, s, (const T *)A,
                           L.ld, L.m, L.n, (const V *)x, axp, rpw, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_residual_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                 int vec, const void *x, double *axp, hipStream_t s) {
    if (vec == VEC_F64) {
        if (dt != RORBK_F64) return hipErrorInvalidValue;
        return resid_typed<double, double>(h, A, aligned, x, axp, s);
    }
    if (dt == RORBK_F32) return resid_typed<float, float>(h, A, aligned, x, axp, s);
    return resid_typed<bf16_t, float>(h, A, aligned, x, axp, s);
}

template <typename T>
static hipError_t gram_typed(const rorbk_handle_s *h, const void *A, const int32_t *idx, int K,
                             double *Gpart, hipStream_t s) {
    const Layout &L = h->L;
    dim3 grid(L.nch_g);
    if (K <= 32)
        hipLaunchKernelGGL((k_gram_dense<T, 2>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    else if (K <= 64)
        hipLaunchKernelGGL((k_gram_dense<T, 4>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_gram_dense<T, 8>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_gram_dense(const rorbk_handle_s *h, const void *A, int dt, const int32_t *idx,
                             int K, double *Gpart, hipStream_t s) {
    if (dt == RORBK_F64) return gram_typed<double>(h, A, idx, K, Gpart, s);
    if (dt == RORBK_F32) return gram_typed<float>(h, A, idx, K, Gpart, s);
    return gram_typed<bf16_t>(h, A, idx, K, Gpart, s);
}

// ------------------------------------------------------------------ setup --
// Centroids (Section 2: the sum of a block's rows), FP64: thread per column,
// rows added in order.  Grid: x = column groups, y = blocks.
template <typename T>
__global__ __launch_bounds__(256) void k_centroid_dense(const T *__restrict__ A, int64_t ld,
                                                        int64_t n, const int64_t *__restrict__ off,
                                                        double *__restrict__ cen) {
    const int64_t t = blockIdx.x;
    const int64_t c = (int64_t)blockIdx.y * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double s = 0.0;
    for (int64_t i = off[t]; i < off[t + 1]; ++i) s += (double)to_v<double>(A[i * ld + c]);
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

// Cosine row sums (Section 2, C(i,j) = |<c_i,c_j>| / (|c_i||c_j|)): a 64 x 64
// tile of the centroid Gram per workgroup (16 x 16 threads, 4 x 4 each, FP64),
// then for each row t of the tile the sum of its 64 normalised |entries| in
// column order -> Sp[t][tile].  A zero centroid has C(t,t) = 1 and C(t,j) = 0.
constexpr int CT = 64;
__global__ __launch_bounds__(256) void k_cos_tiles(const double *__restrict__ cen, int64_t k,
                                                   int64_t n, const double *__restrict__ nrm,
                                                   double *__restrict__ Sp, int64_t ntile) {
    __shared__ double Ti[16][CT + 1], Tj[16][CT + 1];
    __shared__ double outt[CT][CT + 1];
    const int tx = threadIdx.x & 15, ty = threadIdx.x >> 4;
    const int64_t i0 = (int64_t)blockIdx.y * CT, j0 = (int64_t)blockIdx.x * CT;
    double acc[4][4];
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) acc[u][w] = 0.0;
    for (int64_t cb = 0; cb < n; cb += 16) {
        for (int e = threadIdx.x; e < 16 * CT; e += 256) {
            const int r = e / 16, c = e % 16;
            const int64_t col = cb + c;
            Ti[c][r] = (i0 + r < k && col < n) ? cen[(i0 + r) * n + col] : 0.0;
            Tj[c][r] = (j0 + r < k && col < n) ? cen[(j0 + r) * n + col] : 0.0;
        }
        __syncthreads();
#pragma unroll 4
        for (int c = 0; c < 16; ++c) {
            double a[4], bb[4];
#pragma unroll
            for (int u = 0; u < 4; ++u) {
                a[u] = Ti[c][ty * 4 + u];
                bb[u] = Tj[c][tx * 4 + u];
            }
#pragma unroll
            for (int u = 0; u < 4; ++u)
#pragma unroll
                for (int w = 0; w < 4; ++w) acc[u][w] = __builtin_fma(a[u], bb[w], acc[u][w]);
        }
        __syncthreads();
    }
#pragma unroll
    for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int w = 0; w < 4; ++w) {
            const int64_t i = i0 + ty * 4 + u, j = j0 + tx * 4 + w;
            double cij = 0.0;
            if (i < k && j < k) {
                const double ni = nrm[i], nj = nrm[j];
                if (ni == 0.0 || nj == 0.0) cij = (i == j) ? 1.0 : 0.0;
                else cij = fabs(acc[u][w]) / (ni * nj);
            }
            outt[ty * 4 + u][tx * 4 + w] = cij;
        }
    __syncthreads();
    if (threadIdx.x < CT) {
        const int64_t i = i0 + threadIdx.x;
        if (i < k) {
            double s = 0.0;
            for (int w = 0; w < CT; ++w) s += outt[threadIdx.x][w];
            Sp[i * ntile + blockIdx.x] = s;
        }
    }
}

// S_t = sum of the tile partials in tile order, Pbar_t = exp(-2 S_t / n)
// (Section 2, the proposal), and W = running sums of Pbar in block order.
__global__ __launch_bounds__(256) void k_proposal(const double *__restrict__ Sp, int64_t ntile,
                                                  int64_t k, int64_t n, double *__restrict__ S,
                                                  double *__restrict__ pbar,
                                                  double *__restrict__ W) {
    for (int64_t t = threadIdx.x; t < k; t += blockDim.x) {
        double s = 0.0;
        for (int64_t j = 0; j < ntile; ++j) s += Sp[t * ntile + j];
        S[t] = s;
        pbar[t] = exp(-2.0 * s / (double)n);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
        double acc = 0.0;
        for (int64_t t = 0; t < k; ++t) {
            acc += pbar[t];
            W[t] = acc;
        }
    }
}

hipError_t launch_proposal_from_centroids(const rorbk_handle_s *h, double *cen, double *nrm,
                                          double *Sp, hipStream_t s) {
    const Layout &L = h->L;
    hipLaunchKernelGGL(k_rownorm, dim3((unsigned)L.k), dim3(256), 0, s, cen, L.n, nrm);
    const int64_t nt = (L.k + CT - 1) / CT;
    hipLaunchKernelGGL(k_cos_tiles, dim3((unsigned)nt, (unsigned)nt), dim3(256), 0, s, cen, L.k,
                       L.n, nrm, Sp, nt);
    hipLaunchKernelGGL(k_proposal, dim3(1), dim3(256), 0, s, Sp, nt, L.k, L.n, h->d_S,
                       h->d_pbar, h->d_W);
    return hipGetLastError();
}

hipError_t launch_setup_proposal_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                       double *scratch, hipStream_t s) {
    (void)aligned;
    const Layout &L = h->L;
    double *cen = scratch;                      // k * n
    double *nrm = cen + L.k * L.n;              // k
    double *Sp = nrm + L.k;                     // k * ntile
    dim3 grid((unsigned)L.k, (unsigned)((L.n + 255) / 256));
    if (dt == RORBK_F64)
        hipLaunchKernelGGL(k_centroid_dense<double>, grid, dim3(256), 0, s, (const double *)A,
                           L.ld, L.n, h->d_off, cen);
    else if (dt == RORBK_F32)
        hipLaunchKernelGGL(k_centroid_dense<float>, grid, dim3(256), 0, s, (const float *)A, L.ld,
                           L.n, h->d_off, cen);
    else
        hipLaunchKernelGGL(k_centroid_dense<bf16_t>, grid, dim3(256), 0, s, (const bf16_t *)A,
                           L.ld, L.n, h->d_off, cen);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    return launch_proposal_from_centroids(h, cen, nrm, Sp, s);
}

// Stored inverse of each fixed block (Section 3.1 stores the inverse of the
// regularised block Gram): G_t = A_t A_t^T + lambda I in FP64, its packed
// Cholesky factor in LDS, then column j of G_t^{-1} by forward and backward
// substitution (thread j), written row-major (G_t^{-1} is symmetric).
template <typename T, int MT>
__global__ __launch_bounds__(256) void k_block_inverse_dense(const T *__restrict__ A, int64_t ld,
                                                             int64_t n,
                                                             const int64_t *__restrict__ off,
                                                             const int64_t *__restrict__ hoff,
                                                             double lambda, double *__restrict__ H,
                                                             int32_t *__restrict__ fail) {
    __shared__ double At[GT][MAXB + 8];
    __shared__ double Lp[PACKED_MAX];
    __shared__ int64_t rows[MAXB];
    const int64_t t = blockIdx.x;
    const int64_t start = off[t];
    const int K = (int)(off[t + 1] - start);
    for (int q = threadIdx.x; q < K; q += blockDim.x) rows[q] = start + q;
    for (int e = threadIdx.x; e < GT * (MAXB + 8); e += blockDim.x) (&At[0][0])[e] = 0.0;
    __syncthreads();
    const int nt = (K + MT - 1) / MT;
    int bi = -1, bj = -1;
    if ((int)threadIdx.x < nt * (nt + 1) / 2) tile_of(threadIdx.x, nt, &bi, &bj);
    double acc[MT][MT];
    gram_accumulate<T, MT>(A, ld, rows, K, 0, n, acc, bi, bj, At);
    if (bi >= 0) {
#pragma unroll
        for (int u = 0; u < MT; ++u)
#pragma unroll
            for (int w = 0; w < MT; ++w) {
                const int i = bi * MT + u, j = bj * MT + w;
                if (i < K && j <= i) Lp[pk(i, j)] = acc[u][w] + (i == j ? lambda : 0.0);
            }
    }
    __syncthreads();
    if (!chol_packed(Lp, K)) {
        if (threadIdx.x == 0) *fail = 1;
        return;
    }
    double *Hb = H + hoff[t];
    for (int j = threadIdx.x; j < K; j += blockDim.x) {
        double *h = Hb + (int64_t)j * K;
        for (int i = 0; i < K; ++i) {  // L z = e_j
            if (i < j) { h[i] = 0.0; continue; }
            double s = (i == j) ? 1.0 : 0.0;
            for (int q = j; q < i; ++q) s -= Lp[pk(i, q)] * h[q];
            h[i] = s / Lp[pk(i, i)];
        }
        for (int i = K - 1; i >= 0; --i) {  // L^T h = z
            double s = h[i];
            for (int q = i + 1; q < K; ++q) s -= Lp[pk(q, i)] * h[q];
            h[i] = s / Lp[pk(i, i)];
        }
    }
}

hipError_t launch_block_inverses_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                       int32_t *d_fail, hipStream_t s) {
    (void)aligned;
    const Layout &L = h->L;
    const int K = (int)L.bmax;
    dim3 grid((unsigned)L.k);
#define RORBK_INV(T, MT)                                                                    \
    hipLaunchKernelGGL((k_block_inverse_dense<T, MT>), grid, dim3(256), 0, s, (const T *)A, \
                       L.ld, L.n, h->d_off, h->d_hoff, h->lambda, h->d_H, d_fail)
    if (dt == RORBK_F64) {
        if (K <= 32) RORBK_INV(double, 2); else if (K <= 64) RORBK_INV(double, 4); else RORBK_INV(double, 8);
    } else if (dt == RORBK_F32) {
        if (K <= 32) RORBK_INV(float, 2); else if (K <= 64) RORBK_INV(float, 4); else RORBK_INV(float, 8);
    } else {
        if (K <= 32) RORBK_INV(bf16_t, 2); else if (K <= 64) RORBK_INV(bf16_t, 4); else RORBK_INV(bf16_t, 8);
    }
#undef RORBK_INV
    return hipGetLastError();
}

}  // namespace rorbk
