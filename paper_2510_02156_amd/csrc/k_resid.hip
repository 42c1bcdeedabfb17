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
//
// SH (rows whose start is 16-byte aligned or half a vector past it: a 16-byte
// aligned matrix with a row stride of 4 mod 8 elements, BF16 rows of 1000
// bytes for instance): a row that starts half a vector off is read with the
// same aligned 16-byte loads moved back by half a vector, against a second
// copy of x shifted the same way; the vector that would pass the matrix's
// last element takes the element-wise path, and elements outside the row's
// columns are cleared.  The other rows take the aligned form.
template <typename T>
__device__ __forceinline__ uvec4 clear_outside(uvec4 w, int64_t c, int64_t n) {
    constexpr int VW = Tr<T>::VW;
    static_assert(sizeof(T) == 2, "shifted rows: 16-bit values");
#pragma unroll
    for (int e = 0; e < VW / 2; ++e) {
        const int64_t c0 = c + 2 * e, c1 = c0 + 1;
        const uint32_t lo = (c0 >= 0 && c0 < n) ? 0x0000ffffu : 0u;
        const uint32_t hi = (c1 >= 0 && c1 < n) ? 0xffff0000u : 0u;
        w[e] &= (lo | hi);
    }
    return w;
}

// x[c .. c + VW) into registers, zero outside [0, n): 16-byte loads when
// `vec` (x 16-byte aligned and every lane's slice inside [0, n): a
// wave-uniform condition, so that no lane's element loads write registers
// another lane's 16-byte loads are still filling), element loads otherwise.
// c is a multiple of 16 bytes.  Every wave reads its slice of x once, so
// these loads are a sizeable share of the pass's load instructions.
template <typename V, int VW>
__device__ __forceinline__ void x_slice(const V *__restrict__ x, int64_t c, int64_t n, bool vec,
                                        V (&out)[VW]) {
    constexpr int PQ = 16 / sizeof(V);   // elements per 16-byte load
    static_assert(VW % PQ == 0, "whole 16-byte loads per slice");
    if (vec) {
#pragma unroll
        for (int qd = 0; qd < VW / PQ; ++qd) {
            const uvec4 t = *reinterpret_cast<const uvec4 *>(x + c + qd * PQ);
            __builtin_memcpy(&out[qd * PQ], &t, 16);
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) out[e] = (c + e >= 0 && c + e < n) ? x[c + e] : (V)0;
    }
}

// Waves per SIMD at most: FP32 rows of full segments stream fastest with
// three (measured: 114.5 us against 118.9 us with four on the tall 100000 x
// 2000 matrix); the other forms are bounded by their registers.
template <typename T, int SW>
constexpr int resid_waves() { return (sizeof(T) == 4 && SW == SEG) ? 3 : 8; }

template <typename T, typename V, bool AL, int ROWS, int SW, bool SH = false>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, resid_waves<T, SW>())))
void k_resid_dense(const T *__restrict__ A, int64_t ld,
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
    // slice s of the wave covers columns c0 + s * 64 * VW + [0, 64 * VW)
    const bool xal = (reinterpret_cast<uintptr_t>(x) & 15) == 0;
    V xr[NVL][VW];
#pragma unroll
    for (int s = 0; s < NVL; ++s) {
        const int64_t cw = c0 + (int64_t)s * WAVE * VW;
        x_slice<V, VW>(x, cw + (int64_t)lane * VW, n, xal && cw + WAVE * VW <= n, xr[s]);
    }
    V xs[SH ? NVL : 1][VW];   // x moved back by half a vector (SH)
    if constexpr (SH) {
#pragma unroll
        for (int s = 0; s < NVL; ++s) {
            const int64_t cw = c0 + (int64_t)s * WAVE * VW - VW / 2;
            x_slice<V, VW>(x, cw + (int64_t)lane * VW, n, xal && cw >= 0 && cw + WAVE * VW <= n,
                           xs[s]);
        }
    }
    const int64_t last = (m - 1) * ld + n;   // one past the matrix's last element
    const int64_t bx = (int64_t)blockIdx.x - side.jobs;
    const int64_t nwaves = (int64_t)(gridDim.x - side.jobs) * 4;
    const int64_t stride = nwaves * ROWS;
    const uvec4 zero = {0u, 0u, 0u, 0u};
    for (int64_t i = (bx * 4 + w) * ROWS; i < m; i += stride) {
        uvec4 raw[ROWS][NVL];
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            const int64_t row = (i + rr < m) ? i + rr : m - 1;
            if constexpr (SH) {
                // wave-uniform: does this row start half a vector off?
                const int64_t sh = ((row * ld) & (VW - 1)) ? VW / 2 : 0;
#pragma unroll
                for (int s = 0; s < NVL; ++s) {
                    const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW - sh;
                    uvec4 w;
                    if (row * ld + col + VW <= last)
                        w = __builtin_nontemporal_load(
                            reinterpret_cast<const uvec4 *>(A + row * ld + col));
                    else
                        w = load_raw<T, false>(A + row * ld, col, n);
                    raw[rr][s] = clear_outside<T>(w, col, n);
                }
            } else {
#pragma unroll
                for (int s = 0; s < NVL; ++s) {
                    const int64_t col = c0 + (int64_t)(s * WAVE + lane) * VW;
                    raw[rr][s] = load_raw_nt_sel<T, AL>(A + row * ld, col, n, true, A + row * ld, c0);
                }
            }
        }
#pragma unroll
        for (int rr = 0; rr < ROWS; ++rr) {
            V acc = (V)0;
            bool shifted = false;
            if constexpr (SH) {
                const int64_t row = (i + rr < m) ? i + rr : m - 1;
                shifted = ((row * ld) & (VW - 1)) != 0;
            }
#pragma unroll
            for (int s = 0; s < NVL; ++s) {
                V a[VW];
                cvt_raw<T, V>(raw[rr][s], a);
#pragma unroll
                for (int e = 0; e < VW; ++e) acc = fmaT(a[e], shifted ? xs[s][e] : xr[s][e], acc);
            }
            const V sres = group_sum(acc, WAVE);
            if (lane == 0 && i + rr < m) axp[seg * m + i + rr] = (double)sres;
        }
    }
}

template <typename T, typename V, int ROWS, int SW, bool SH = false>
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
    if constexpr (SH) {
        hipLaunchKernelGGL((k_resid_dense<T, V, false, ROWS, SW, true>), grid, dim3(256), 0, s,
                           (const T *)A, L.ld, L.m, L.n, (const V *)x, axp,
                           (const Ctrl *)h->d_ctrl, side);
        return hipGetLastError();
    }
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
    // BF16 rows that start 16-byte aligned or half a vector past it (a
    // 16-byte aligned matrix, row stride 4 mod 8 elements): the shifted form
    const bool sh = !aligned && (reinterpret_cast<uintptr_t>(A) & 15) == 0 && (h->L.ld & 7) == 4;
    if (n <= 512)
        return sh ? resid_typed<bf16_t, float, 16, 512, true>(h, A, aligned, x, axp, side, s)
                  : resid_typed<bf16_t, float, 16, 512>(h, A, aligned, x, axp, side, s);
    if (n <= 1024)
        return sh ? resid_typed<bf16_t, float, 8, 1024, true>(h, A, aligned, x, axp, side, s)
                  : resid_typed<bf16_t, float, 8, 1024>(h, A, aligned, x, axp, side, s);
    return sh ? resid_typed<bf16_t, float, 4, SEG, true>(h, A, aligned, x, axp, side, s)
              : resid_typed<bf16_t, float, 4, SEG>(h, A, aligned, x, axp, side, s);
}

}  // namespace rorbk
