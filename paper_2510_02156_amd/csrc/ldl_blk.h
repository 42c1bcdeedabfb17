// ldl_blk.h -- the greedy block system of Algorithm 1, (G + lambda I) y = r_I
// for a greedy set of at most 64 rows, solved on one wave by an LDL^T
// factorisation in 16-column panels whose trailing updates run on FP64 MFMA.
// Internal to the library; used by the greedy kernels of k_common.hip and
// k_fwd.hip.
#pragma once

#include <utility>

#include "rorbk_device.h"

namespace rorbk {

constexpr int LB_RS = 65;   // row stride of the work matrix S (64 x 65 doubles)

// Elimination step k of one 16-column panel (columns c0 .. c0 + 15, rows
// c0 .. N - 1).  Lane i holds row c0 + i of the panel, a[0..15] (on the
// panel's diagonal block only the entries j <= i mean anything), and z_{c0+i}.
// The pivot d_k comes from lane k; 1 / d_k is the hardware reciprocal with
// one Newton step, the second folded into its uses (l = a r1 + a r1 (1 -
// d r1)), and the next pivot is formed straight from this one, d_{k+1} =
// a_{k+1,k+1} - a_{k+1,k}^2 / d_k.  Rows below the pivot take l_ik = a_ik / d_k,
// a_ij -= l_ik a_jk for the panel columns j > k and z_i -= l_ik z_k; the a_jk
// are read from col, where every lane published its a_ik, and column k + 1 is
// published right after its own update.  The factor goes to S as it is
// formed: l_ik below the diagonal and d_k on it (lower triangle, row-major),
// and the unscaled a_ik of the rows below the diagonal block (the columns of
// L D the trailing update needs) transposed into the free upper triangle,
// S[c0 + k][c0 + i].  Stores that carry nothing (lanes past the last row,
// rows of the diagonal block for the transposed copy) go to the unused 65th
// column of S, so that no store needs a branch.
template <int N, int k>
__device__ __forceinline__ void lb_step(double (&a)[16], double &zi, double &dnext, int lane,
                                        int c0, bool live, double *S, double *colbuf, bool &ok) {
    const double *col = colbuf + (k & 1) * 64;
    double *nxt = colbuf + ((k + 1) & 1) * 64;
    const double d = bcast64(dnext, k);
    ok = ok && (d > 0.0);
    const double r0 = __builtin_amdgcn_rcp(d);
    const double e0 = __builtin_fma(-d, r0, 1.0);
    const double r1 = __builtin_fma(r0, e0, r0);
    const double e1 = __builtin_fma(-d, r1, 1.0);
    const double akk = a[k];
    const double m1 = akk * r1;
    const double c = __builtin_fma(m1, e1, m1);
    if constexpr (k + 1 < 16) {
        const double t = akk * akk;
        const double tr1 = t * r1;
        const double u = __builtin_fma(-t, r1, a[k + 1]);
        dnext = __builtin_fma(-tr1, e1, u);
    }
    const double zk = bcast64(zi, k);
    zi = (lane > k) ? __builtin_fma(-c, zk, zi) : zi;
    const int pad = lane * LB_RS + 64;
    S[live ? (c0 + lane) * LB_RS + c0 + k : pad] = (lane > k) ? c : d;
    S[(live && lane >= 16) ? (c0 + k) * LB_RS + c0 + lane : pad] = akk;
    double cv[16];
#pragma unroll
    for (int j = k + 1; j < 16; ++j) cv[j] = col[j];
    if constexpr (k + 1 < 16) {
        a[k + 1] = __builtin_fma(-c, cv[k + 1], a[k + 1]);
        nxt[lane] = a[k + 1];
    }
#pragma unroll
    for (int j = k + 2; j < 16; ++j) a[j] = __builtin_fma(-c, cv[j], a[j]);
    __builtin_amdgcn_wave_barrier();
}

template <int N, int... Ks>
__device__ __forceinline__ void lb_steps(std::integer_sequence<int, Ks...>, double (&a)[16],
                                         double &zi, int lane, int c0, bool live, double *S,
                                         double *colbuf, bool &ok) {
    double dnext = a[0];
    (lb_step<N, Ks>(a, zi, dnext, lane, c0, live, S, colbuf, ok), ...);
}

// Trailing update of panel c0 on MFMA: S_IJ -= L_I (L D)_J^T for the 16 x 16
// sub-tiles (I, J), J <= I, of rows and columns c0 + 16 .. N - 1, four
// v_mfma_f64_16x16x4f64 per sub-tile (panel columns in order); L_I from the
// lower triangle, (L D)_J from the transposed copy in the upper triangle.
// Diagonal sub-tiles are written whole (their upper halves are never read).
template <int N, int C0>
__device__ __forceinline__ void lb_update(double *S) {
    constexpr int NB = (N - C0 - 16) / 16;
    const int lane = threadIdx.x & 63, li = lane & 15, lk = lane >> 4;
#pragma unroll
    for (int I = 0; I < NB; ++I)
#pragma unroll
        for (int J = 0; J <= I; ++J) {
            const int rI = C0 + 16 + 16 * I, cJ = C0 + 16 + 16 * J;
            dvec4 acc;
#pragma unroll
            for (int r = 0; r < 4; ++r) acc[r] = S[(rI + lk + 4 * r) * LB_RS + cJ + li];
#pragma unroll
            for (int k0 = 0; k0 < 16; k0 += 4) {
                const double av = -S[(rI + li) * LB_RS + C0 + k0 + lk];
                const double bv = S[(C0 + k0 + lk) * LB_RS + cJ + li];
                acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av, bv, acc, 0, 0, 0);
            }
#pragma unroll
            for (int r = 0; r < 4; ++r) S[(rI + lk + 4 * r) * LB_RS + cJ + li] = acc[r];
        }
}

template <int N, int P>
__device__ __forceinline__ void lb_panel(double *S, double *z, double *colbuf, bool &ok) {
    constexpr int C0 = 16 * P;
    const int lane = threadIdx.x & 63;
    const bool live = lane < N - C0;   // lanes holding a row of the panel
    const int row = C0 + (live ? lane : 0);
    double a[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = (j <= lane) ? S[row * LB_RS + C0 + j] : 0.0;
    double zi = live ? z[row] : 0.0;
    colbuf[lane] = a[0];
    __builtin_amdgcn_wave_barrier();
    lb_steps<N>(std::make_integer_sequence<int, 16>{}, a, zi, lane, C0, live, S, colbuf, ok);
    if (live) z[row] = zi;
    __builtin_amdgcn_wave_barrier();
    if constexpr (C0 + 16 < N) {
        lb_update<N, C0>(S);
        __builtin_amdgcn_wave_barrier();
    }
}

template <int N, int... Ps>
__device__ __forceinline__ void lb_panels(std::integer_sequence<int, Ps...>, double *S, double *z,
                                          double *colbuf, bool &ok) {
    (lb_panel<N, Ps>(S, z, colbuf, ok), ...);
}

// Entry f of the packed lower triangle (row-major, j <= i) of the padded
// system written into S: the Gram value g (plus lambda on the diagonal) for
// rows below K, the identity from row K on.  Every f < 64 * 65 / 2 is written
// once by whichever thread holds it, so the workgroup fills S in parallel.
__device__ __forceinline__ void lb_put(double *S, int f, double g, int K, double lambda) {
    int i = (int)((sqrtf(8.0f * (float)f + 1.0f) - 1.0f) * 0.5f);
    while (i * (i + 1) / 2 > f) --i;
    while ((i + 1) * (i + 2) / 2 <= f) ++i;
    const int j = f - i * (i + 1) / 2;
    S[i * LB_RS + j] = (i < K) ? ((i == j) ? g + lambda : g) : ((i == j) ? 1.0 : 0.0);
}

// Broadcast of lane J of each 16-lane row to the whole row (DPP row_newbcast).
template <int J>
__device__ __forceinline__ double lb_rowbc(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xf, 0xf, false);
}

// Step k of the backward pass within one 16-row block: y_k is final in lane k
// of every 16-lane row; rows i < k of the block take w_i -= l_ki y_k.
template <int k>
__device__ __forceinline__ void lb_back_step(double &w, const double (&lv)[16], int li) {
    const double yk = lb_rowbc<k>(w);
    w = (li < k) ? __builtin_fma(-lv[k], yk, w) : w;
}

template <int... Ks>
__device__ __forceinline__ void lb_back_steps(std::integer_sequence<int, Ks...>, double &w,
                                              const double (&lv)[16], int li) {
    (lb_back_step<15 - Ks>(w, lv, li), ...);
}

// Backward pass y = L^{-T} w over the 16-row block P (rows c0 .. c0 + 15), w
// in wb (LDS, N entries): every 16-lane row of the wave solves the block's
// unit upper-triangular system L_PP^T y_P = w_P (lane li holding row c0 + li,
// l_ki of its column preloaded), then the rows above the block take
// w_i -= sum_k l_{c0+k, i} y_{c0+k}, k in order.
template <int P>
__device__ __forceinline__ void lb_back_block(const double *S, double *wb) {
    constexpr int C0 = 16 * P;
    const int lane = threadIdx.x & 63, li = lane & 15;
    double lv[16];
#pragma unroll
    for (int k = 0; k < 16; ++k) lv[k] = (k > li) ? S[(C0 + k) * LB_RS + C0 + li] : 0.0;
    double w = wb[C0 + li];
    lb_back_steps(std::make_integer_sequence<int, 16>{}, w, lv, li);
    __builtin_amdgcn_wave_barrier();
    if (lane < 16) wb[C0 + lane] = w;
    __builtin_amdgcn_wave_barrier();
    if constexpr (C0 > 0) {
        const int i = lane < C0 ? lane : 0;
        double lc[16], yv[16];
#pragma unroll
        for (int k = 0; k < 16; ++k) {
            lc[k] = S[(C0 + k) * LB_RS + i];
            yv[k] = wb[C0 + k];
        }
        double acc = wb[i];
#pragma unroll
        for (int k = 0; k < 16; ++k) acc = __builtin_fma(-lc[k], yv[k], acc);
        __builtin_amdgcn_wave_barrier();
        if (lane < C0) wb[lane] = acc;
        __builtin_amdgcn_wave_barrier();
    }
}

template <int... Ps>
__device__ __forceinline__ void lb_back_blocks(std::integer_sequence<int, Ps...>, const double *S,
                                               double *wb) {
    constexpr int NP = sizeof...(Ps);
    (lb_back_block<NP - 1 - Ps>(S, wb), ...);
}

// Single-wave solve of the padded N x N system (N = 16, 32 or 64) held
// in S (the 64 x 65 work matrix, lower triangle of rows 0 .. N - 1, filled by
// lb_put: the Gram with lambda on the diagonal, the identity from row K on),
// right-hand side in z (entries K .. N - 1 zero; overwritten by y), colbuf
// 2 x 64 doubles.  The identity beyond K leaves the leading K x K factor and
// solution unchanged.  LDL^T by 16-column panels (forward substitution inside
// them), then y = L^{-T} D^{-1} z by 16-row blocks from the last.  S ends
// holding L below the diagonal and D on it.  No block barrier inside: the
// workgroup's other waves may be elsewhere.  Returns false if a pivot is not
// positive.
template <int N>
__device__ __forceinline__ bool ldl_blk(double *S, double *z, double *colbuf) {
    const int lane = threadIdx.x & 63;
    bool ok = true;
    lb_panels<N>(std::make_integer_sequence<int, N / 16>{}, S, z, colbuf, ok);
    if (!ok) return false;
    if (lane < N) z[lane] = z[lane] / S[lane * LB_RS + lane];
    __builtin_amdgcn_wave_barrier();
    lb_back_blocks(std::make_integer_sequence<int, N / 16>{}, S, z);
    return true;
}

// K <= 64 on one wave: the smallest padded size that holds the system.
__device__ __forceinline__ bool ldl_blk64(double *S, double *z, int K, double *colbuf /* 2 x 64 */) {
    if (K <= 16) return ldl_blk<16>(S, z, colbuf);
    if (K <= 32) return ldl_blk<32>(S, z, colbuf);
    return ldl_blk<64>(S, z, colbuf);
}

}  // namespace rorbk
