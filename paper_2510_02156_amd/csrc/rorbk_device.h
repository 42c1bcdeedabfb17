// rorbk_device.h -- device-side building blocks shared by the ROR-BK kernels:
// element types, 16-byte vector loads, deterministic wave reductions and the
// packed lower-triangular Cholesky used for every block Gram.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "rorbk_internal.h"

namespace rorbk {

constexpr int WAVE = 64;
constexpr int MAXB = RORBK_MAX_BLOCK_ROWS + 1;          // largest block (rows)
constexpr int PACKED_MAX = MAXB * (MAXB + 1) / 2;       // packed lower size

typedef uint16_t bf16_t;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef uint32_t uvec4 __attribute__((ext_vector_type(4)));

// Storage traits: elements per 16-byte load.
template <typename T> struct Tr;
template <> struct Tr<double> { static constexpr int VW = 2; };
template <> struct Tr<float> { static constexpr int VW = 4; };
template <> struct Tr<bf16_t> { static constexpr int VW = 8; };

__device__ __forceinline__ float bf16_to_f32(bf16_t v) {
    return __uint_as_float(((uint32_t)v) << 16);
}

template <typename V> __device__ __forceinline__ V to_v(double a) { return (V)a; }
template <typename V> __device__ __forceinline__ V to_v(float a) { return (V)a; }
template <typename V> __device__ __forceinline__ V to_v(bf16_t a) { return (V)bf16_to_f32(a); }

__device__ __forceinline__ double fmaT(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fmaT(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

// Load VW consecutive elements starting at column c of a row (converted to V).
// ALIGNED: the row start is 16-byte aligned and c is a multiple of VW, so a
// full vector is one 16-byte load; the ragged tail (c + VW > n) is read
// element by element with zeros past n.
template <typename T, typename V, bool ALIGNED>
__device__ __forceinline__ void load_vec(const T *__restrict__ row, int64_t c, int64_t n,
                                         V (&out)[Tr<T>::VW]) {
    constexpr int VW = Tr<T>::VW;
    if (ALIGNED && c + VW <= n) {
        if constexpr (sizeof(T) == 8) {
            double2 v = *reinterpret_cast<const double2 *>(row + c);
            out[0] = (V)v.x;
            out[1] = (V)v.y;
        } else if constexpr (sizeof(T) == 4) {
            float4 v = *reinterpret_cast<const float4 *>(row + c);
            out[0] = (V)v.x; out[1] = (V)v.y; out[2] = (V)v.z; out[3] = (V)v.w;
        } else {
            uint4 v = *reinterpret_cast<const uint4 *>(row + c);
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                out[2 * e] = (V)__uint_as_float(w[e] << 16);
                out[2 * e + 1] = (V)__uint_as_float(w[e] & 0xffff0000u);
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) out[e] = (c + e < n) ? to_v<V>(row[c + e]) : (V)0;
    }
}

// Streaming variant for the residual pass: A is read once per pass, so the
// loads carry the non-temporal hint.
template <typename T, typename V, bool ALIGNED>
__device__ __forceinline__ void load_vec_nt(const T *__restrict__ row, int64_t c, int64_t n,
                                            V (&out)[Tr<T>::VW]) {
    constexpr int VW = Tr<T>::VW;
    if (ALIGNED && c + VW <= n) {
        if constexpr (sizeof(T) == 8) {
            dvec2 v = __builtin_nontemporal_load(reinterpret_cast<const dvec2 *>(row + c));
            out[0] = (V)v.x;
            out[1] = (V)v.y;
        } else if constexpr (sizeof(T) == 4) {
            fvec4 v = __builtin_nontemporal_load(reinterpret_cast<const fvec4 *>(row + c));
            out[0] = (V)v.x; out[1] = (V)v.y; out[2] = (V)v.z; out[3] = (V)v.w;
        } else {
            uvec4 v = __builtin_nontemporal_load(reinterpret_cast<const uvec4 *>(row + c));
            uint32_t w[4] = {v.x, v.y, v.z, v.w};
#pragma unroll
            for (int e = 0; e < 4; ++e) {
                out[2 * e] = (V)__uint_as_float(w[e] << 16);
                out[2 * e + 1] = (V)__uint_as_float(w[e] & 0xffff0000u);
            }
        }
    } else {
#pragma unroll
        for (int e = 0; e < VW; ++e) out[e] = (c + e < n) ? to_v<V>(row[c + e]) : (V)0;
    }
}

// Butterfly sum over the `width` lanes of a lane group (width a power of two
// <= 64).  The combination order is fixed, so the result is reproducible.
template <typename V>
__device__ __forceinline__ V group_sum(V v, int width) {
    for (int off = width >> 1; off > 0; off >>= 1) v += __shfl_xor(v, off, width);
    return v;
}

// Sum over a workgroup of `nthreads` threads in a fixed order: butterfly
// within waves, then wave partials summed in wave order.  `sh` holds at least
// nthreads/64 doubles.  All threads receive the result.
__device__ __forceinline__ double block_sum(double v, double *sh) {
    v = group_sum(v, WAVE);
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    __syncthreads();
    if (lane == 0) sh[w] = v;
    __syncthreads();
    double s = 0.0;
    const int nw = (blockDim.x + 63) >> 6;
    for (int i = 0; i < nw; ++i) s += sh[i];
    __syncthreads();
    return s;
}

__device__ __forceinline__ int pk(int i, int j) { return i * (i + 1) / 2 + j; }  // j <= i

// In-place Cholesky of a packed lower K x K matrix in LDS by the whole
// workgroup, one barrier per elimination step.  Step k updates the trailing
// triangle with the unscaled pivot column (G_ij -= G_ik G_jk / G_kk); the
// columns are scaled by 1/sqrt(pivot) at the end.  Returns false (uniformly)
// if a pivot is not positive.
__device__ inline bool chol_packed(double *Lp, int K) {
    __shared__ int s_bad;
    if (threadIdx.x == 0) s_bad = 0;
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        const double d = Lp[pk(k, k)];
        if (!(d > 0.0)) {
            if (threadIdx.x == 0) s_bad = 1;
            break;  // uniform: every thread reads the same pivot
        }
        const double inv = 1.0 / d;
        const int w = K - k - 1;
        const int tot = w * (w + 1) / 2;
        for (int f = threadIdx.x; f < tot; f += blockDim.x) {
            // f -> (a, b) with b <= a < w, row-major over the packed triangle
            int a = (int)((sqrtf(8.0f * (float)f + 1.0f) - 1.0f) * 0.5f);
            while (a * (a + 1) / 2 > f) --a;
            while ((a + 1) * (a + 2) / 2 <= f) ++a;
            const int b = f - a * (a + 1) / 2;
            const int i = k + 1 + a, j = k + 1 + b;
            Lp[pk(i, j)] -= Lp[pk(i, k)] * (Lp[pk(j, k)] * inv);
        }
        __syncthreads();
    }
    __syncthreads();
    const bool bad = s_bad != 0;
    if (bad) return false;
    // scale: L_ik = G_ik / sqrt(d_k) for i >= k
    const int tot = K * (K + 1) / 2;
    for (int f = threadIdx.x; f < tot; f += blockDim.x) {
        int i = (int)((sqrtf(8.0f * (float)f + 1.0f) - 1.0f) * 0.5f);
        while (i * (i + 1) / 2 > f) --i;
        while ((i + 1) * (i + 2) / 2 <= f) ++i;
        const int k = f - i * (i + 1) / 2;
        const double dk = Lp[pk(k, k)];
        // the diagonal is rewritten last, after every column entry has used it
        if (i != k) Lp[f] = Lp[f] / sqrt(dk);
    }
    __syncthreads();
    for (int k = threadIdx.x; k < K; k += blockDim.x) Lp[pk(k, k)] = sqrt(Lp[pk(k, k)]);
    __syncthreads();
    return true;
}

// y = (L L^T)^{-1} r with L packed lower in LDS; done by wave 0 (lane p holds
// entries p, p+64, p+128), no barriers inside.  r and y live in LDS (may alias).
__device__ inline void chol_solve_wave(const double *Lp, int K, const double *r, double *y) {
    if (threadIdx.x >= WAVE) return;
    const int lane = threadIdx.x;
    double v[3];
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int i = lane + 64 * s;
        v[s] = (i < K) ? r[i] : 0.0;
    }
    // forward: L z = r
    for (int j = 0; j < K; ++j) {
        const int s = j >> 6, src = j & 63;
        double vj = (s == 0) ? v[0] : (s == 1 ? v[1] : v[2]);
        vj = __shfl(vj, src, WAVE);
        const double zj = vj / Lp[pk(j, j)];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int i = lane + 64 * t;
            if (i > j && i < K) v[t] -= Lp[pk(i, j)] * zj;
            if (i == j) v[t] = zj;
        }
    }
    // backward: L^T y = z
    for (int j = K - 1; j >= 0; --j) {
        const int s = j >> 6, src = j & 63;
        double vj = (s == 0) ? v[0] : (s == 1 ? v[1] : v[2]);
        vj = __shfl(vj, src, WAVE);
        const double yj = vj / Lp[pk(j, j)];
#pragma unroll
        for (int t = 0; t < 3; ++t) {
            const int i = lane + 64 * t;
            if (i < j) v[t] -= Lp[pk(j, i)] * yj;
            if (i == j) v[t] = yj;
        }
    }
#pragma unroll
    for (int s = 0; s < 3; ++s) {
        const int i = lane + 64 * s;
        if (i < K) y[i] = v[s];
    }
}

}  // namespace rorbk
