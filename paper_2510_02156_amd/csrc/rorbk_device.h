// rorbk_device.h -- device-side building blocks shared by the ROR-BK kernels:
// element types, 16-byte vector loads, deterministic wave reductions and the
// packed lower-triangular Cholesky used for every block Gram.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <utility>

#include "rorbk_internal.h"

namespace rorbk {

constexpr int WAVE = 64;
constexpr int MAXB = RORBK_MAX_BLOCK_ROWS + 1;          // largest block (rows)
constexpr int PACKED_MAX = MAXB * (MAXB + 1) / 2;       // packed lower size
constexpr int BIGB = RORBK_MAX_BIG_BLOCK_ROWS;          // largest block, dense large-block path
constexpr int MAXK = BIGB > MAXB ? BIGB : MAXB;         // largest greedy set

typedef uint16_t bf16_t;
typedef double dvec2 __attribute__((ext_vector_type(2)));
typedef float fvec4 __attribute__((ext_vector_type(4)));
typedef uint32_t uvec4 __attribute__((ext_vector_type(4)));
typedef double dvec4 __attribute__((ext_vector_type(4)));

// Closed-form partition (Algorithm 1, first step): block t starts at
// t*q + min(t, rem) and has q or q+1 rows; its stored inverse starts at
// sum_{s<t} b_s^2.
__device__ __forceinline__ int64_t blk_start(int64_t t, int64_t q, int64_t rem) {
    return t * q + (t < rem ? t : rem);
}
__device__ __forceinline__ int blk_rows(int64_t t, int64_t q, int64_t rem) {
    return (int)(q + (t < rem ? 1 : 0));
}
__device__ __forceinline__ int64_t blk_hoff(int64_t t, int64_t q, int64_t rem) {
    const int64_t big = t < rem ? t : rem;
    return big * (q + 1) * (q + 1) + (t - big) * q * q;
}

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

// Elements of a raw 16-byte vector (VW elements from column c) at or past
// `lim` set to zero, by selects (no branch).
template <typename T>
__device__ __forceinline__ uvec4 mask_raw(uvec4 w, int64_t c, int64_t lim) {
    if constexpr (sizeof(T) == 8) {
        const bool k1 = c + 1 < lim;
        const bool k0 = c < lim;
        w[0] = k0 ? w[0] : 0u;
        w[1] = k0 ? w[1] : 0u;
        w[2] = k1 ? w[2] : 0u;
        w[3] = k1 ? w[3] : 0u;
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) w[e] = (c + e < lim) ? w[e] : 0u;
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            const uint32_t lo = (c + 2 * e < lim) ? 0x0000ffffu : 0u;
            const uint32_t hi = (c + 2 * e + 1 < lim) ? 0xffff0000u : 0u;
            w[e] &= (lo | hi);
        }
    }
    return w;
}

// 16 raw bytes (VW elements) of a row at column c (c < lim); elements at or
// past `lim` read as zero.  ALIGNED (row start 16-byte aligned, row stride a
// multiple of VW elements, c a multiple of VW): one 16-byte load, which stays
// inside the row's stride even when it crosses lim (c < lim <= n <= stride),
// and the tail masked by selects, so the code has no branch around the load.
// Otherwise a full vector whose address is 8-byte aligned (rows of 16- or
// 32-bit values whose stride is a multiple of 8 bytes) is read as two 8-byte
// loads, anything else element by element.
template <typename T, bool ALIGNED>
__device__ __forceinline__ uvec4 load_raw(const T *__restrict__ row, int64_t c, int64_t lim) {
    constexpr int VW = Tr<T>::VW;
    if constexpr (ALIGNED) return mask_raw<T>(*reinterpret_cast<const uvec4 *>(row + c), c, lim);
    if constexpr (!ALIGNED && sizeof(T) < 8) {
        if (c + VW <= lim && (reinterpret_cast<uintptr_t>(row + c) & 7) == 0) {
            const uint2 lo = *reinterpret_cast<const uint2 *>(row + c);
            const uint2 hi = *reinterpret_cast<const uint2 *>(row + c + VW / 2);
            const uvec4 v = {lo.x, lo.y, hi.x, hi.y};
            return v;
        }
    }
    uvec4 w = {0u, 0u, 0u, 0u};
    if constexpr (sizeof(T) == 8) {
#pragma unroll
        for (int e = 0; e < 2; ++e)
            if (c + e < lim) {
                const uint64_t u = (uint64_t)__double_as_longlong((double)row[c + e]);
                w[2 * e] = (uint32_t)u;
                w[2 * e + 1] = (uint32_t)(u >> 32);
            }
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e)
            if (c + e < lim) w[e] = __float_as_uint((float)row[c + e]);
    } else {
#pragma unroll
        for (int e = 0; e < 8; ++e)
            if (c + e < lim) w[e >> 1] |= ((uint32_t)(uint16_t)row[c + e]) << (16 * (e & 1));
    }
    return w;
}

// As load_raw, with the full 16-byte load marked non-temporal (streamed
// once, not kept in the caches).
template <typename T, bool ALIGNED>
__device__ __forceinline__ uvec4 load_raw_nt(const T *__restrict__ row, int64_t c, int64_t lim) {
    if constexpr (ALIGNED)
        return mask_raw<T>(__builtin_nontemporal_load(reinterpret_cast<const uvec4 *>(row + c)),
                           c, lim);
    return load_raw<T, ALIGNED>(row, c, lim);
}

// load_raw of (row, c) when `ok` and c < lim, else zero, with no branch
// around the load: otherwise the vector at (srow, sc) is read instead (any
// vector known to lie inside the matrix, sc < lim) and dropped by a select.
// (A load behind a lane-dependent branch makes the compiler wait for it to
// land before the other lanes' zero may be written to the same registers,
// which turns loads meant to overlap into a chain of memory round trips.)
template <typename T, bool ALIGNED>
__device__ __forceinline__ uvec4 load_raw_sel(const T *__restrict__ row, int64_t c, int64_t lim,
                                              bool ok, const T *__restrict__ srow, int64_t sc) {
    const bool g = ok && c < lim;
    const uvec4 w = load_raw<T, ALIGNED>(g ? row : srow, g ? c : sc, lim);
    const uvec4 z = {0u, 0u, 0u, 0u};
    return g ? w : z;
}

template <typename T, bool ALIGNED>
__device__ __forceinline__ uvec4 load_raw_nt_sel(const T *__restrict__ row, int64_t c, int64_t lim,
                                                 bool ok, const T *__restrict__ srow, int64_t sc) {
    const bool g = ok && c < lim;
    const uvec4 w = load_raw_nt<T, ALIGNED>(g ? row : srow, g ? c : sc, lim);
    const uvec4 z = {0u, 0u, 0u, 0u};
    return g ? w : z;
}

template <typename T, typename V>
__device__ __forceinline__ void cvt_raw(const uvec4 &w, V (&out)[Tr<T>::VW]) {
    if constexpr (sizeof(T) == 8) {
        out[0] = (V)__longlong_as_double((long long)(((uint64_t)w[1] << 32) | w[0]));
        out[1] = (V)__longlong_as_double((long long)(((uint64_t)w[3] << 32) | w[2]));
    } else if constexpr (sizeof(T) == 4) {
#pragma unroll
        for (int e = 0; e < 4; ++e) out[e] = (V)__uint_as_float(w[e]);
    } else {
#pragma unroll
        for (int e = 0; e < 4; ++e) {
            out[2 * e] = (V)__uint_as_float(w[e] << 16);
            out[2 * e + 1] = (V)__uint_as_float(w[e] & 0xffff0000u);
        }
    }
}

// FP64 MFMA tile of a Gram product: acc += X_a X_b^T over columns [c0, c1)
// for a 16 x 16 tile, one wave.  Lane l supplies row ra (A side) and rb (B
// side) for tile row/column l % 16 (a negative row reads as zero) and the
// E = 32 / sizeof(T) >= 4 consecutive columns c + g*E .. of lane group
// g = l / 16, which serve as the k index of E v_mfma_f64_16x16x4f64 steps
// (the sum runs over every column once, in a fixed order).  Result layout:
// D[i][j] sits in register i / 4 of lane (i % 4) * 16 + j.  c0 must be a
// multiple of E when ALIGNED.
template <typename T, bool ALIGNED>
__device__ __forceinline__ void mfma_gram_tile(const T *__restrict__ X, int64_t ld, int64_t ra,
                                               int64_t rb, int64_t c0, int64_t c1, dvec4 &acc) {
    constexpr int VW = Tr<T>::VW;
    constexpr int E = (sizeof(T) == 8) ? 4 : VW;   // columns per lane per macro step
    constexpr int NL = E / VW;                      // 16-byte loads per row per step
    constexpr int U = 4;                            // macro steps in flight
    const int g = (threadIdx.x & 63) >> 4;
    const T *pa = X + (ra >= 0 ? ra : 0) * ld;
    const T *pb = X + (rb >= 0 ? rb : 0) * ld;
    const bool same = (ra == rb);
    for (int64_t c = c0; c < c1; c += 4 * E * U) {
        uvec4 wa[U][NL], wb[U][NL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t col = c + (int64_t)u * 4 * E + (int64_t)g * E;
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                wa[u][h] = load_raw_sel<T, ALIGNED>(pa, col + h * VW, c1, ra >= 0, X, c0);
                wb[u][h] = load_raw_sel<T, ALIGNED>(pb, col + h * VW, c1, !same && rb >= 0, X, c0);
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                double av[VW], bv[VW];
                cvt_raw<T, double>(wa[u][h], av);
                if (same) {
#pragma unroll
                    for (int e = 0; e < VW; ++e) bv[e] = av[e];
                } else {
                    cvt_raw<T, double>(wb[u][h], bv);
                }
#pragma unroll
                for (int e = 0; e < VW; ++e)
                    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(av[e], bv[e], acc, 0, 0, 0);
            }
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

// t-th tile of the lower triangle of an nt x nt tile grid, row-major.
__device__ __forceinline__ void tile_of(int t, int nt, int *bi, int *bj) {
    int i = 0, base = 0;
    while (i < nt && base + i + 1 <= t) { base += i + 1; ++i; }
    if (i >= nt) { *bi = -1; *bj = -1; return; }
    *bi = i;
    *bj = t - base;
}

// Symmetric positive definite solve (G + diag) y = r for K <= MAXB in one
// workgroup of 256 threads, G given packed lower in LDS (Gp, overwritten),
// r in LDS (z, overwritten by y).  Factorisation G = L D L^T (unit L) by
// right-looking elimination: thread t keeps one MT x MT tile of the lower
// triangle in registers; at step k the owners of column k publish it to LDS
// (double-buffered), and after one barrier everyone applies the rank-1 update
// a_ij -= g_ik g_jk / d_k, which also carries the right-hand side through the
// forward substitution.  Column k is kept in Gp (unscaled) for the backward
// substitution y_k = z_k / d_k - sum_{i>k} (g_ik / d_k) y_i, run by wave 0.
// Returns false (uniformly) if a pivot d_k is not positive.
template <int MT>
__device__ bool ldl_solve(double *Gp, double *z, int K, double *colbuf /* 2*MAXB */) {
    __shared__ int s_bad;
    const int nt = (K + MT - 1) / MT;
    int bi = -1, bj = -1;
    if ((int)threadIdx.x < nt * (nt + 1) / 2) tile_of(threadIdx.x, nt, &bi, &bj);
    double a[MT][MT];
#pragma unroll
    for (int u = 0; u < MT; ++u)
#pragma unroll
        for (int v = 0; v < MT; ++v) {
            const int i = bi * MT + u, j = bj * MT + v;
            a[u][v] = (bi >= 0 && i < K && j <= i) ? Gp[pk(i, j)] : 0.0;
        }
    if (threadIdx.x == 0) s_bad = 0;
    // column 0 comes straight from Gp
    for (int i = threadIdx.x; i < K; i += blockDim.x) colbuf[i] = Gp[pk(i, 0)];
    __syncthreads();
    for (int k = 0; k < K; ++k) {
        const double *col = colbuf + (k & 1) * MAXB;
        double *nxt = colbuf + ((k + 1) & 1) * MAXB;
        const double d = col[k];
        if (!(d > 0.0)) {
            if (threadIdx.x == 0) s_bad = 1;
            break;  // uniform: every thread reads the same pivot
        }
        const double inv = 1.0 / d;
        // right-hand side (forward substitution with unit L)
        const double zk = z[k];
        if (bi >= 0) {
            double ci[MT], cj[MT];
#pragma unroll
            for (int u = 0; u < MT; ++u) {
                const int i = bi * MT + u, j = bj * MT + u;
                ci[u] = (i > k && i < K) ? col[i] : 0.0;
                cj[u] = (j > k && j < K) ? col[j] * inv : 0.0;
            }
#pragma unroll
            for (int u = 0; u < MT; ++u)
#pragma unroll
                for (int v = 0; v < MT; ++v) a[u][v] = __builtin_fma(-ci[u], cj[v], a[u][v]);
            // publish column k+1 (owners: tiles whose column block holds k+1)
            const int kk = k + 1;
            if (kk < K && kk / MT == bj) {
#pragma unroll
                for (int u = 0; u < MT; ++u) {
                    const int i = bi * MT + u;
#pragma unroll
                    for (int v = 0; v < MT; ++v)
                        if (bj * MT + v == kk && i >= kk && i < K) nxt[i] = a[u][v];
                }
            }
        }
        // keep column k (unscaled) for the backward pass; update z
        for (int i = k + threadIdx.x; i < K; i += blockDim.x) {
            Gp[pk(i, k)] = col[i];
            if (i > k) z[i] = __builtin_fma(-col[i] * inv, zk, z[i]);
        }
        __syncthreads();
    }
    __syncthreads();
    if (s_bad) return false;
    // backward: y_k = z_k / d_k - sum_{i>k} (g_ik / d_k) y_i, column oriented
    if (threadIdx.x < WAVE) {
        const int lane = threadIdx.x;
        double w[3], invd[3];
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int i = lane + 64 * s;
            invd[s] = (i < K) ? 1.0 / Gp[pk(i, i)] : 0.0;
            w[s] = (i < K) ? z[i] * invd[s] : 0.0;
        }
        for (int k = K - 1; k >= 0; --k) {
            const int s = k >> 6, src = k & 63;
            double yk = (s == 0) ? w[0] : (s == 1 ? w[1] : w[2]);
            yk = __shfl(yk, src, WAVE);
#pragma unroll
            for (int t = 0; t < 3; ++t) {
                const int i = lane + 64 * t;
                if (i < k) w[t] = __builtin_fma(-Gp[pk(k, i)] * invd[t], yk, w[t]);
            }
        }
#pragma unroll
        for (int s = 0; s < 3; ++s) {
            const int i = lane + 64 * s;
            if (i < K) z[i] = w[s];
        }
    }
    __syncthreads();
    return true;
}

// Broadcast lane `src` (wave-uniform) of a double to the whole wave.
__device__ __forceinline__ double bcast64(double v, int src) {
    const long long u = __double_as_longlong(v);
    const int lo = __builtin_amdgcn_readlane((int)(u & 0xffffffffLL), src);
    const int hi = __builtin_amdgcn_readlane((int)(u >> 32), src);
    return __longlong_as_double(((long long)hi << 32) | (unsigned int)lo);
}

}  // namespace rorbk
