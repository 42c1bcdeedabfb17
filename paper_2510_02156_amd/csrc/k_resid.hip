// k_resid.hip -- the full residual pass of ROR-BK for a dense row-major
// matrix (FP64, FP32 or BF16 storage): the one kernel that streams all of A
// every outer iteration, and so the one bound by HBM bandwidth.
#include "rorbk_device.h"
#include "xgram.h"

namespace rorbk {

constexpr int SEG = 2048;  // columns of one residual segment (x kept in VGPRs)

// ------------------------------------------------------------ residual pass --
// Algorithm 1, r = b - A x: the products (A x)_i over one 2048-column segment
// (SW columns of it when the whole matrix is narrower, SW = 512 or 1024).
// A grid of a few workgroups per CU walks the rows: wave w takes rows
// w*ROWS .. w*ROWS+ROWS-1, then the same rows plus nwaves*ROWS, and so on.
// For each group of ROWS rows every 16-byte load of the group is issued
// (non-temporal, raw bytes) before any of them is converted or used, so each
// wave keeps ROWS * SW * sizeof(T) bytes in flight (narrow matrices take more
// rows at a time); then each row's lane sums (FMA in column order) are
// combined by a fixed butterfly.  Each lane keeps its entries of x in
// registers.  Rows past the end re-read the last row (in bounds) and discard
// the result.  axp[seg][i] = partial (A x)_i; the selection kernel subtracts
// the segment sum from b.  Grid: x = workgroups, y = segments.  The first
// side.jobs workgroups of segment row 0 instead form the cross-Gram tiles of
// the next iteration's sampled blocks (xgram.h): MFMA work on a few rows that
// sits in cache, done while the pass streams A (those workgroups of the other
// segment rows leave at once).
template <typename T, typename V, bool AL, int ROWS, int SW>
__global__ __launch_bounds__(256) void k_resid_dense(const T *__restrict__ A, int64_t ld,
                                                     int64_t m, int64_t n,
                                                     const V *__restrict__ x,
                                                     double *__restrict__ axp,
                                                     const Ctrl *__restrict__ ctrl, XgSide side) {
    if (ctrl && ctrl->done) return;
    if ((int)blockIdx.x < side.jobs) {
        if (blockIdx.y == 0)
            xgram_tile<T, AL>(A, ld, n, side.tau, side.ti, side.q, side.rem, side.bmax,
                              (int)blockIdx.x, side.out);
        return;
    }
    constexpr int VW = Tr<T>::VW;
    constexpr int NVL = SW / (WAVE * VW);
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
    const int64_t bx = (int64_t)blockIdx.x - side.jobs;
    const int64_t nwaves = (int64_t)(gridDim.x - side.jobs) * 4;
    const int64_t stride = nwaves * ROWS;
    const uvec4 zero = {0u, 0u, 0u, 0u};
    for (int64_t i = (bx * 4 + w) * ROWS; i < m; i += stride) {
        uvec4 raw[ROWS][NVL];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            const int64_t row = (i + rr < m) ? i + rr : m - 1;
#pragma unroll
            for (int s = 0; s < NVL; ++s) {
                const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW;
                raw[rr][s] = load_raw_nt_sel<T, AL>(A + row * ld, col, n, true, A + row * ld, c0);
            }
        }
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            V acc = (V)0;
#pragma unroll
            for (int s = 0; s < NVL; ++s) {
                V a[VW];
                cvt_raw<T, V>(raw[rr][s], a);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc = fmaT(a[e], xr[s][e], acc);
            }
            const V sres = group_sum(acc, WAVE);
            if (lane == 0 && i + rr < m) axp[seg * m + i + rr] = (double)sres;
        }
    }
}

template <typename T, typename V, int ROWS, int SW>
static hipError_t resid_typed(const rorbk_handle_s *h, const void *A, int aligned,
                              const void *x, double *axp, const XgSide &side, hipStream_t s) {
    static_assert(SW == SEG || SW == 512 || SW == 1024, "segment width");
    const Layout &L = h->L;
    // grid over all segments: 16 workgroups per CU for FP32 and FP64 rows of
    // full 2048-column segments (more than are resident at once: the later
    // ones fill in as the first finish, which evens out the tail), as long as
    // every wave still takes at least 3 row groups (each wave loads its slice
    // of x once); 2 per CU otherwise (BF16 and narrow rows are slower with
    // more); fewer for short matrices
    constexpr int PER_CU = (SW == SEG && sizeof(T) >= 4) ? 16 : 2;
    int64_t groups = (L.m + 4 * ROWS - 1) / (4 * ROWS);
    int64_t cap = PER_CU * (int64_t)h->ncu / L.nseg;
    if (PER_CU > 2) {
        int64_t c3 = L.m / (4 * ROWS * 3);
        const int64_t c2 = 2 * (int64_t)h->ncu / L.nseg;
        if (c3 < c2) c3 = c2;
        if (cap > c3) cap = c3;
    }
    if (cap < 1) cap = 1;
    if (groups > cap) groups = cap;
    dim3 grid((unsigned)(groups + side.jobs), (unsigned)L.nseg);
    if (aligned)
        hipLaunchKernelGGL((k_resid_dense<T, V, true, ROWS, SW>), grid, dim3(256), 0, s, (const T *)A,
                           L.ld, L.m, L.n, (const V *)x, axp, (const Ctrl *)h->d_ctrl, side);
    else
        hipLaunchKernelGGL((k_resid_dense<T, V, false, ROWS, SW>), grid, dim3(256), 0, s,
                           (const T *)A, L.ld, L.m, L.n, (const V *)x, axp,
                           (const Ctrl *)h->d_ctrl, side);
    return hipGetLastError();
}

// About sixteen 16-byte loads in flight per wave: rows per group chosen from
// the loads one row takes (the segment width over 64 lanes x 16 bytes).
hipError_t launch_residual_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                 int vec, const void *x, double *axp, hipStream_t s) {
    const XgSide none = {nullptr, 0, 0, 0, 0, 0, nullptr};
    return launch_residual_dense_side(h, A, dt, aligned, vec, x, axp, none, s);
}

hipError_t launch_residual_dense_side(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                      int vec, const void *x, double *axp, const XgSide &side,
                                      hipStream_t s) {
    const int64_t n = h->L.n;
    if (vec == VEC_F64) {
        if (dt != RORBK_F64) return hipErrorInvalidValue;
        if (n <= 512) return resid_typed<double, double, 4, 512>(h, A, aligned, x, axp, side, s);
        if (n <= 1024) return resid_typed<double, double, 2, 1024>(h, A, aligned, x, axp, side, s);
        // the unaligned FP64 form needs twice the registers per row in flight
        if (aligned) return resid_typed<double, double, 2, SEG>(h, A, aligned, x, axp, side, s);
        return resid_typed<double, double, 1, SEG>(h, A, aligned, x, axp, side, s);
    }
    if (dt == RORBK_F32) {
        if (n <= 512) return resid_typed<float, float, 8, 512>(h, A, aligned, x, axp, side, s);
        if (n <= 1024) return resid_typed<float, float, 4, 1024>(h, A, aligned, x, axp, side, s);
        return resid_typed<float, float, 2, SEG>(h, A, aligned, x, axp, side, s);
    }
    if (n <= 512) return resid_typed<bf16_t, float, 16, 512>(h, A, aligned, x, axp, side, s);
    if (n <= 1024) return resid_typed<bf16_t, float, 8, 1024>(h, A, aligned, x, axp, side, s);
    return resid_typed<bf16_t, float, 4, SEG>(h, A, aligned, x, axp, side, s);
}

}  // namespace rorbk
