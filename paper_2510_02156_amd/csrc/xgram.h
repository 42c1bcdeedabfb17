// xgram.h -- cross-Grams of the three blocks an outer iteration samples, for
// the fused sampled steps of k_fwd.hip; included by k_fwd.hip (stand-alone
// launch), k_resid.hip (spare workgroups of the residual pass) and
// k_common.hip (spare workgroups of the selection), which run the same
// arithmetic for the same wave count.
#pragma once

#include "rorbk_device.h"

namespace rorbk {

constexpr int FWD_B = RORBK_FWD_MAX_BLOCK;   // largest block (rows) of the fused-step path

// ------------------------------------------------------------ cross-Grams --
// Tile job `job` of the cross-Grams of the blocks drawn at tau[ti .. ti+2]:
// pair 0 = A_2 A_1^T, pair 1 = A_3 A_1^T, pair 2 = A_3 A_2^T (0-based block
// order 1, 2, 3), each split into 16 x 16 tiles (nb = ceil(bmax / 16) per
// side).  The NW waves of the workgroup take equal shares of the columns (in
// multiples of the MFMA step) and their tiles are added in wave order; out
// holds [3][bmax][bmax] doubles, entry (i, j) = <row i of the row block,
// row j of the column block> at out[j * bmax + i] (column-major, so that the
// consumers' loads over i are contiguous).  Used both stand-alone and by spare
// workgroups of the residual pass; the arithmetic is the same either way.
template <typename T, bool AL, int NW = 4>
__device__ __forceinline__ void xgram_tile(const T *__restrict__ A, int64_t ld, int64_t n,
                           const int32_t *__restrict__ tau, int64_t ti, int64_t q, int64_t rem,
                           int bmax, int job, double *__restrict__ out) {
    constexpr int E = (sizeof(T) == 8) ? 4 : Tr<T>::VW;
    const int nb = (bmax + 15) / 16;
    const int pair = job / (nb * nb), rest = job - pair * nb * nb;
    const int bi = rest / nb, bj = rest - bi * nb;
    const int la = (pair == 0) ? 1 : 2, lb = (pair == 2) ? 1 : 0;
    const int64_t ta = tau[ti + la], tb = tau[ti + lb];
    const int64_t sa = blk_start(ta, q, rem), sb = blk_start(tb, q, rem);
    const int ca = blk_rows(ta, q, rem), cb = blk_rows(tb, q, rem);
    if (bi * 16 >= ca || bj * 16 >= cb) return;   // uniform: a tile past both blocks' rows
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15;
    const int64_t stepc = 4 * E;
    const int64_t span = ((n + NW * stepc - 1) / (NW * stepc)) * stepc;
    const int64_t wa = (int64_t)w * span;
    const int64_t wb = (wa + span < n) ? wa + span : n;
    const int64_t ra = (bi * 16 + li < ca) ? sa + bi * 16 + li : -1;
    const int64_t rb = (bj * 16 + li < cb) ? sb + bj * 16 + li : -1;
    dvec4 acc = {0.0, 0.0, 0.0, 0.0};
    if (wa < wb) mfma_gram_tile<T, AL>(A, ld, ra, rb, wa, wb, acc);
    __shared__ double red[NW][64][4];
#pragma unroll
    for (int r = 0; r < 4; ++r) red[w][lane][r] = acc[r];
    __syncthreads();
    if (w == 0) {
        double *o = out + (int64_t)pair * bmax * bmax;
#pragma unroll
        for (int r = 0; r < 4; ++r) {
            double s = red[0][lane][r];
#pragma unroll
            for (int v = 1; v < NW; ++v) s += red[v][lane][r];
            const int ii = bi * 16 + (lane >> 4) + 4 * r, jj = bj * 16 + li;
            if (ii < ca && jj < cb) o[jj * bmax + ii] = s;
        }
    }
}

// Number of tile jobs of the cross-Grams for blocks of at most bmax rows.
__host__ __device__ inline int xgram_jobs(int bmax) {
    const int nb = (bmax + 15) / 16;
    return 3 * nb * nb;
}

}  // namespace rorbk
