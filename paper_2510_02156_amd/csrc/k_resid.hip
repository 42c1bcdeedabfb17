// k_resid.hip -- the full residual pass of ROR-BK for a dense row-major
// matrix (FP64, FP32 or BF16 storage): the one kernel that streams all of A
// every outer iteration, and so the one bound by HBM bandwidth.
#include "rorbk_device.h"

namespace rorbk {

constexpr int SEG = 2048;  // columns of one residual segment (x kept in VGPRs)

// ------------------------------------------------------------ residual pass --
// Algorithm 1, r = b - A x: the products (A x)_i over one 2048-column segment.
// A persistent grid (a few workgroups per CU) walks the rows: wave w takes rows
// w*ROWS, w*ROWS + nwaves*ROWS, ..., ROWS rows in flight at a time.  Each lane
// keeps its 32 entries of x in registers and streams the row with 16-byte
// non-temporal loads; lane sums are combined by a fixed butterfly.
// axp[seg][i] = partial (A x)_i; the selection kernel subtracts the segment sum
// from b.  Grid: x = workgroups, y = segments.
template <typename T, typename V, bool AL, int ROWS>
__global__ __launch_bounds__(256) void k_resid_dense(const T *__restrict__ A, int64_t ld,
                                                     int64_t m, int64_t n,
                                                     const V *__restrict__ x,
                                                     double *__restrict__ axp,
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
    const int64_t nwaves = (int64_t)gridDim.x * 4;
    const int64_t stride = nwaves * ROWS;
    for (int64_t i = ((int64_t)blockIdx.x * 4 + w) * ROWS; i < m; i += stride) {
        V acc[ROWS];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) acc[rr] = (V)0;
#pragma unroll
        for (int s = 0; s < NVL; ++s) {
            const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW;
#pragma unroll
            for (int rr = 0; rr < ROWS; ++rr) {
                if (i + rr < m && col < n) {
                    V a[VW];
                    load_vec_nt<T, V, AL>(A + (i + rr) * ld, col, n, a);
#pragma unroll
                    for (int e = 0; e < VW; ++e) acc[rr] = fmaT(a[e], xr[s][e], acc[rr]);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            const V sres = group_sum(acc[rr], WAVE);
            if (lane == 0 && i + rr < m) axp[seg * m + i + rr] = (double)sres;
        }
    }
}

template <typename T, typename V, int ROWS>
static hipError_t resid_typed(const rorbk_handle_s *h, const void *A, int aligned,
                              const void *x, double *axp, hipStream_t s) {
    const Layout &L = h->L;
    // persistent grid: 4 workgroups (16 waves) per CU, fewer for short matrices
    int64_t groups = (L.m + 4 * ROWS - 1) / (4 * ROWS);
    const int64_t cap = 4 * (int64_t)h->ncu;
    if (groups > cap) groups = cap;
    dim3 grid((unsigned)groups, (unsigned)L.nseg);
    if (aligned)
        hipLaunchKernelGGL((k_resid_dense<T, V, true, ROWS>), grid, dim3(256), 0, s, (const T *)A,
                           L.ld, L.m, L.n, (const V *)x, axp, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_resid_dense<T, V, false, ROWS>), grid, dim3(256), 0, s,
                           (const T *)A, L.ld, L.m, L.n, (const V *)x, axp,
                           (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_residual_dense(const rorbk_handle_s *h, const void *A, int dt, int aligned,
                                 int vec, const void *x, double *axp, hipStream_t s) {
    if (vec == VEC_F64) {
        if (dt != RORBK_F64) return hipErrorInvalidValue;
        return resid_typed<double, double, 1>(h, A, aligned, x, axp, s);
    }
    if (dt == RORBK_F32) return resid_typed<float, float, 2>(h, A, aligned, x, axp, s);
    return resid_typed<bf16_t, float, 2>(h, A, aligned, x, axp, s);
}

}  // namespace rorbk
