// gram_tiles.h -- one 64 x 64 tile of a Gram matrix X_S X_S^T on FP64 MFMA,
// for the block Grams of the setup (Algorithm 1, the stored inverses) and the
// greedy Gram of large greedy sets.  Internal to the library.
#pragma once

#include "rorbk_device.h"

namespace rorbk {

// Accumulates, for one 64 x 64 tile (row groups a = rows pa[0..3], b = rows
// pb[0..3], 16 rows each, lane li = threadIdx % 16 holding row li of each
// group), the 16 sub-tile products over the columns [c0, c1) of the rows in
// four waves: wave w takes a contiguous quarter of the range (a multiple of
// 4 E columns), lane group g = lane / 16 takes E columns of every 4 E, so
// each v_mfma_f64_16x16x4f64 sums 4 columns and the products are summed in
// column-step order.  This is the order of the 16 x 16 tile kernels, so a
// sub-tile gets the same value from either.  Every row value loaded feeds
// four products (the lower ten on a diagonal tile, `same`).  Whole macro steps
// load unconditionally (callers point rows past the end, va / vb false, at a
// valid row: their products only reach outputs that are not written); the
// last partial step takes the guarded loads.  acc is in the MFMA layout:
// element (i, j) of sub-tile (s, t) in register i / 4 of lane (i % 4) 16 + j.
// U2: two macro steps of FP64 rows in flight (the contiguous rows of a block
// Gram; measured faster there, slower on the gathered rows of a greedy Gram).
template <typename T, bool AL, bool U2 = false>
__device__ __forceinline__ void gram64_accumulate(const T *const (&pa)[4], const T *const (&pb)[4],
                                                  const bool (&va)[4], const bool (&vb)[4],
                                                  bool same, int64_t c0, int64_t c1,
                                                  dvec4 (&acc)[4][4]) {
    constexpr int VW = Tr<T>::VW;
    constexpr int E = (sizeof(T) == 8) ? 4 : VW;   // columns per lane per macro step
    constexpr int NL = E / VW;                      // 16-byte loads per row per step
    constexpr int U = (sizeof(T) == 8 && !U2) ? 1 : 2;   // macro steps in flight
    const int w = threadIdx.x >> 6, g = (threadIdx.x & 63) >> 4;
    const int64_t stepc = 4 * E;
    const int64_t span = ((c1 - c0 + 4 * stepc - 1) / (4 * stepc)) * stepc;
    const int64_t wa = c0 + w * span;
    const int64_t wb = (wa + span < c1) ? wa + span : c1;
    const dvec4 z4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2) acc[s2][t2] = z4;
    const uvec4 zu = {0u, 0u, 0u, 0u};
    for (int64_t c = wa; c < wb; c += 4 * E * U) {
        const bool whole = AL && (c + 4 * E * U <= wb);   // wave-uniform
        uvec4 xa[U][4][NL], xb[U][4][NL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t col = c + (int64_t)u * 4 * E + (int64_t)g * E;
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const int64_t cc = col + h * VW;
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) {
                    if (whole) {
                        xa[u][s2][h] = *reinterpret_cast<const uvec4 *>(pa[s2] + cc);
                        xb[u][s2][h] = same ? zu : *reinterpret_cast<const uvec4 *>(pb[s2] + cc);
                    } else {
                        // rows are valid even where va / vb are false
                        xa[u][s2][h] = load_raw_sel<T, AL>(pa[s2], cc, wb, va[s2], pa[s2], wa);
                        xb[u][s2][h] = load_raw_sel<T, AL>(pb[s2], cc, wb, !same && vb[s2], pb[s2], wa);
                    }
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                double av[4][VW], bv[4][VW];
#pragma unroll
                for (int s2 = 0; s2 < 4; ++s2) cvt_raw<T, double>(xa[u][s2][h], av[s2]);
                if (same) {
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                        for (int e = 0; e < VW; ++e) bv[s2][e] = av[s2][e];
                } else {
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2) cvt_raw<T, double>(xb[u][s2][h], bv[s2]);
                }
#pragma unroll
                for (int e = 0; e < VW; ++e)
#pragma unroll
                    for (int s2 = 0; s2 < 4; ++s2)
#pragma unroll
                        for (int t2 = 0; t2 < 4; ++t2)
                            if (!same || t2 <= s2)
                                acc[s2][t2] = __builtin_amdgcn_mfma_f64_16x16x4f64(
                                    av[s2][e], bv[t2][e], acc[s2][t2], 0, 0, 0);
            }
    }
}

// The four waves' accumulators of tile (bi, bj) summed in wave order through
// LDS (one row of sub-tiles at a time, wave w summing sub-tile column w) and
// written packed lower, out[pk(i, j)] for i < K, j <= i.  Contains barriers:
// the whole workgroup calls it.
__device__ __forceinline__ void gram64_store(const dvec4 (&acc)[4][4], int bi, int bj, int K,
                                             double *__restrict__ out) {
    __shared__ double red[4][16][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        if (s2 > 0) __syncthreads();   // the previous row's sums are read
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][t2 * 4 + r][lane] = acc[s2][t2][r];
        __syncthreads();
        const int t2 = w;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q2 = t2 * 4 + r;
            const double v = ((red[0][q2][lane] + red[1][q2][lane]) + red[2][q2][lane]) +
                             red[3][q2][lane];
            const int ii = bi * 64 + s2 * 16 + (lane >> 4) + 4 * r;
            const int jj = bj * 64 + t2 * 16 + li;
            if (ii < K && jj <= ii) out[pk(ii, jj)] = v;
        }
    }
}

// The four waves' accumulators summed in wave order, as in gram64_store, and
// the whole 64 x 64 tile written row-major, out[i * 64 + j] (on a diagonal
// tile, `same` in gram64_accumulate, the sub-tiles above the diagonal hold
// zeros).  Contains barriers: the whole workgroup calls it.
__device__ __forceinline__ void gram64_store_tile(const dvec4 (&acc)[4][4],
                                                  double *__restrict__ out) {
    __shared__ double red[4][16][64];
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        if (s2 > 0) __syncthreads();
#pragma unroll
        for (int t2 = 0; t2 < 4; ++t2)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][t2 * 4 + r][lane] = acc[s2][t2][r];
        __syncthreads();
        const int t2 = w;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            const int q2 = t2 * 4 + r;
            const double v = ((red[0][q2][lane] + red[1][q2][lane]) + red[2][q2][lane]) +
                             red[3][q2][lane];
            const int ii = s2 * 16 + (lane >> 4) + 4 * r;
            out[ii * 64 + t2 * 16 + li] = v;
        }
    }
}

}  // namespace rorbk
