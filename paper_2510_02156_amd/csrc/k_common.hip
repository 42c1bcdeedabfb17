// k_common.hip -- format-independent ROR-BK kernels: partition, sampler,
// norms, residual-driven selection (per-block norms, stop test, top-K) and the
// greedy block's Cholesky solve.
#include "ldl_blk.h"
#include "rorbk_device.h"
#include "xgram.h"

namespace rorbk {

// ------------------------------------------------------------- partition --
// Algorithm 1, first step: k contiguous blocks of floor(m/k) rows, the first
// (m mod k) of them one row longer.  hoff[t] = sum_{s<t} b_s^2 locates the
// stored inverse of block t.
__global__ void k_partition(int64_t m, int64_t k, int64_t *off, int64_t *hoff) {
    const int64_t t = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (t > k) return;
    const int64_t q = m / k, rem = m - k * q;
    off[t] = t * q + (t < rem ? t : rem);
    const int64_t big = (t < rem ? t : rem);
    hoff[t] = big * (q + 1) * (q + 1) + (t - big) * q * q;
}

hipError_t launch_partition(int64_t m, int64_t k, int64_t *off, int64_t *hoff,
                            hipStream_t s) {
    const int64_t nb = (k + 1 + 255) / 256;
    hipLaunchKernelGGL(k_partition, dim3((unsigned)nb), dim3(256), 0, s, m, k, off, hoff);
    return hipGetLastError();
}

// --------------------------------------------------------------- sampler --
// SplitMix64 (Steele, Lea and Flood, OOPSLA 2014), counter form: word c of a
// seed is the generator's output finaliser applied to seed + (c+1)*0x9E37..15.
__device__ __forceinline__ uint64_t splitmix_word(uint64_t seed, uint64_t c) {
    uint64_t z = seed + (c + 1) * 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    return z ^ (z >> 31);
}

// Draw l of outer iteration j (Algorithm 1, inner loop; proposal of Section 2):
// u = top 53 bits of word 3j + l - 1 scaled to [0,1); the block is the number
// of running sums W_t not exceeding u * W_{k-1} (inverse CDF of
// P = Pbar / sum Pbar), at most k - 1.
__global__ void k_sample(uint64_t seed, int64_t j0, int64_t count, const double *__restrict__ W,
                         int64_t k, int32_t *__restrict__ tau) {
    const int64_t d = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (d >= 3 * count) return;
    const int64_t it = d / 3;
    const int l = (int)(d - 3 * it);
    const uint64_t w = splitmix_word(seed, (uint64_t)(3 * (j0 + it) + l));
    const double u = (double)(w >> 11) * 0x1.0p-53;
    const double target = u * W[k - 1];
    // W is non-decreasing: count of W_t <= target by binary search
    int64_t lo = 0, hi = k;
    while (lo < hi) {
        const int64_t mid = (lo + hi) >> 1;
        if (W[mid] <= target) lo = mid + 1; else hi = mid;
    }
    tau[d] = (int32_t)(lo > k - 1 ? k - 1 : lo);
}

hipError_t launch_sample(uint64_t seed, int64_t j0, int64_t count, const double *W,
                         int64_t k, int32_t *tau, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    const int64_t nb = (3 * count + 255) / 256;
    hipLaunchKernelGGL(k_sample, dim3((unsigned)nb), dim3(256), 0, s, seed, j0, count, W, k, tau);
    return hipGetLastError();
}

__global__ void k_copy_i32(const int32_t *src, int32_t *dst, int64_t count) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < count) dst[i] = src[i];
}

hipError_t launch_copy_tau(const int32_t *src, int32_t *dst, int64_t count, hipStream_t s) {
    if (count <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_copy_i32, dim3((unsigned)((count + 255) / 256)), dim3(256), 0, s,
                       src, dst, count);
    return hipGetLastError();
}

// ----------------------------------------------------------------- norms --
// ||v||^2 in a fixed order: one workgroup, thread t summing entries t,
// t + 1024, ... in order (each load instruction reads consecutive entries,
// eight in flight per thread), then the workgroup sum.
template <typename V>
__global__ __launch_bounds__(1024) void k_norm2(const V *__restrict__ v, int64_t len,
                                                double *__restrict__ out) {
    __shared__ double sh[16];
    constexpr int U = 8;
    const int64_t st = blockDim.x;
    double s = 0.0;
    int64_t i = threadIdx.x;
    for (; i + (U - 1) * st < len; i += U * st) {
        double t[U];
#pragma unroll
        for (int u = 0; u < U; ++u) t[u] = (double)v[i + u * st];
#pragma unroll
        for (int u = 0; u < U; ++u) s = __builtin_fma(t[u], t[u], s);
    }
    for (; i < len; i += st) {
        const double t = (double)v[i];
        s = __builtin_fma(t, t, s);
    }
    s = block_sum(s, sh);
    if (threadIdx.x == 0) *out = s;
}

hipError_t launch_norm2(const void *v, int vec, int64_t len, double *red, double *out,
                        hipStream_t s) {
    (void)red;
    if (vec == VEC_F64)
        hipLaunchKernelGGL(k_norm2<double>, dim3(1), dim3(1024), 0, s, (const double *)v, len, out);
    else
        hipLaunchKernelGGL(k_norm2<float>, dim3(1), dim3(1024), 0, s, (const float *)v, len, out);
    return hipGetLastError();
}

// -------------------------------------------------------------- selection --
// Keys order |r_i|: the IEEE bits of |r_i| (sign cleared) are monotone in
// |r_i| and hence in r_i^2 (Algorithm 1, greedy step), without rounding a
// square.  Ties go to the lower index.
__device__ __forceinline__ uint64_t key_of(double v) {
    return (uint64_t)__double_as_longlong(v) & 0x7fffffffffffffffULL;
}
__device__ __forceinline__ uint64_t key_of(float v) {
    return (uint64_t)(__float_as_uint(v) & 0x7fffffffu);
}

constexpr int SEL_T = 512;          // threads of the selection kernels
constexpr int SEL_CHUNK = 4096;     // rows per selection chunk (upper bound)
constexpr int SEL_MERGE = 8192;     // candidates per merge workgroup
constexpr int SEL_BPC = 256;        // blocks per selection chunk (upper bound)

// Inclusive prefix sum of a 32-bit count over the 64 lanes of a wave, lane 0
// first: sums within each row of 16 lanes by row_shr 1, 2, 4, 8 (lanes that
// would read from outside their row add 0), then rows 1 and 3 add the last
// lane of rows 0 and 2 (row_bcast:15) and rows 2 and 3 the last lane of row 1
// (row_bcast:31).  Integer sums, so the order of the additions is immaterial.
__device__ __forceinline__ uint32_t wave_prefix_sum_u32(uint32_t x) {
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false);
    x += (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false);
    return x;
}

// Largest 32-bit value over the 64 lanes of a wave, in every lane: the
// prefix maximum by the same DPP steps as wave_prefix_sum_u32 (0 is the
// identity), read from the last lane.
__device__ __forceinline__ uint32_t wave_max_u32(uint32_t x) {
    uint32_t t;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x111, 0xf, 0xf, false); x = t > x ? t : x;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x112, 0xf, 0xf, false); x = t > x ? t : x;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x114, 0xf, 0xf, false); x = t > x ? t : x;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x118, 0xf, 0xf, false); x = t > x ? t : x;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x142, 0xa, 0xf, false); x = t > x ? t : x;
    t = (uint32_t)__builtin_amdgcn_update_dpp(0, (int)x, 0x143, 0xc, 0xf, false); x = t > x ? t : x;
    return (uint32_t)__builtin_amdgcn_readlane((int)x, 63);
}

// Largest and smallest of a per-thread 32-bit value over the workgroup: DPP
// steps within each wave (the smallest as the complement of the largest
// complement), then the per-wave results through LDS.  Every thread receives
// both.  Contains one __syncthreads.
__device__ __forceinline__ void block_minmax_u32(uint32_t mx, uint32_t mn, uint32_t *omx,
                                                 uint32_t *omn) {
    __shared__ uint32_t wmx[16], wmn[16];
    mx = wave_max_u32(mx);
    mn = ~wave_max_u32(~mn);
    const int w = threadIdx.x >> 6, nw = blockDim.x >> 6;
    if ((threadIdx.x & 63) == 0) { wmx[w] = mx; wmn[w] = mn; }
    __syncthreads();
    uint32_t a = wmx[0], c = wmn[0];
    for (int i = 1; i < nw; ++i) {
        a = wmx[i] > a ? wmx[i] : a;
        c = wmn[i] < c ? wmn[i] : c;
    }
    *omx = a;
    *omn = c;
}

// Radix select over the N >= K keys that the workgroup holds in registers:
// element i = threadIdx.x + u * SEL_T is kv[u] of its thread (u < PER; every
// histogram pass reads registers, not LDS).  The 32-bit view (key >> shift) of the
// largest and the smallest key (vmax, vmin, from block_minmax_u32) share
// their leading bits with every key, so the search starts at the highest bit
// where the two differ and spends no pass on a common prefix.  Digits of up to
// 8 bits follow, most significant first: finds a masked threshold (T, mask)
// and the number `need` of elements whose masked key equals T that complete
// the top K (elements with a larger masked key are all in).  Stops as soon as
// the boundary bucket holds exactly `need` elements.  One barrier per pass:
// every wave reads the whole histogram and finds the boundary bin itself (the
// same result in every wave), and each pass also clears the next pass's
// histogram: three in rotation, so that one was last read two passes back,
// which every wave finished before the previous pass's barrier.
template <int PER>
__device__ __forceinline__ void radix_select(const uint64_t (&kv)[PER], int N, int K, int shift,
                                             uint32_t vmax, uint32_t vmin, uint64_t *T_out,
                                             uint64_t *mask_out, int *need_out) {
    static_assert(SEL_T >= 256, "one thread per bin clears a histogram");
    __shared__ uint32_t hist[3][256];
    const uint32_t dv = vmax ^ vmin;
    if (dv == 0 && shift == 0) {  // all keys equal: the first K by index
        *T_out = (uint64_t)vmax;
        *mask_out = ~0ull;
        *need_out = K;
        return;
    }
    // highest differing bit (bit shift - 1 if the views agree)
    const int top = dv ? shift + 31 - __clz((int)dv) : shift - 1;
    const uint64_t pm = ~((2ull << top) - 1ull);
    uint64_t prefix = ((uint64_t)vmax << shift) & pm, mask = pm;
    int need = K;
    const int lane = threadIdx.x & 63;
    if (threadIdx.x < 256) hist[0][threadIdx.x] = 0u;
    __syncthreads();
    int p = 0;
    for (int hi = top; hi >= 0; hi -= 8) {
        const int lo = hi >= 7 ? hi - 7 : 0;
        const uint64_t dmask = (1ull << (hi - lo + 1)) - 1ull;
        uint32_t *H = hist[p];
        const int pn = (p == 2) ? 0 : p + 1;
        if (threadIdx.x < 256) hist[pn][threadIdx.x] = 0u;
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * SEL_T;
            if (i < N && ((kv[u] ^ prefix) & mask) == 0)
                atomicAdd(&H[(kv[u] >> lo) & dmask], 1u);
        }
        __syncthreads();
        p = pn;
        // lane l holds bins 4 (63 - l) .. 4 (63 - l) + 3, so the prefix sum
        // over lanes counts the elements in bins >= 4 (63 - l)
        uint32_t h[4];
        uint32_t ls = 0;
#pragma unroll
        for (int u = 0; u < 4; ++u) { h[u] = H[4 * (63 - lane) + u]; ls += h[u]; }
        const uint32_t pre = wave_prefix_sum_u32(ls);
        const unsigned long long bal = __ballot(pre >= (uint32_t)need);
        if (bal == 0ull) continue;   // (not reached: N >= K)
        const int fl = __ffsll((long long)bal) - 1;   // the lowest lane reaching `need`
        uint32_t above = (uint32_t)__builtin_amdgcn_readlane((int)pre, fl) -
                         (uint32_t)__builtin_amdgcn_readlane((int)ls, fl);
        uint32_t hf[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) hf[u] = (uint32_t)__builtin_amdgcn_readlane((int)h[u], fl);
        int bin = 4 * (63 - fl);
        uint32_t inbin = hf[0];
        for (int u = 3; u >= 0; --u) {
            if (above + hf[u] >= (uint32_t)need) { bin = 4 * (63 - fl) + u; inbin = hf[u]; break; }
            above += hf[u];
        }
        need -= (int)above;
        prefix |= (uint64_t)bin << lo;
        mask |= dmask << lo;
        if (inbin == (uint32_t)need) break;
    }
    *T_out = prefix;
    *mask_out = mask;
    *need_out = need;
}

// Emit, in ascending index order, every element whose masked key exceeds T
// and the first `need` elements whose masked key equals T (K in total).
// Element i = threadIdx.x + u * NT is kv[u] (and iv[u] with IDS, else its
// position i) of its thread, so index order is (round, wave, lane): ranks
// within a wave come from ballots, and the counts of earlier (round, wave)
// pairs from one scan over their totals.  Outputs get base added to the index.
template <int NT, int ROUNDS, bool IDS>
__device__ __forceinline__ void compact_topk(const uint64_t (&kv)[ROUNDS],
                                             const int32_t (&iv)[ROUNDS], int N, int K,
                                             uint64_t T, uint64_t mask, int need, uint64_t *okey,
                                             int32_t *oidx, int32_t base) {
    constexpr int NW = NT / 64, NS = ROUNDS * NW;
    static_assert(NS <= 128, "one scan lane holds two (round, wave) totals");
    // totals per (round, wave): greater-than count << 16 | equal count
    // (each at most N <= 8192, so neither half carries into the other)
    __shared__ uint32_t wcnt[NS];
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    // per round: rank among the wave's "greater" lanes (bits 0..7), among its
    // "equal" lanes (bits 8..15), and the two flags (bits 16, 17)
    uint32_t rk[ROUNDS];
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
        const int i = threadIdx.x + u * NT;
        const uint64_t mk = kv[u] & mask;
        const bool gt = (i < N) && mk > T, eq = (i < N) && mk == T;
        const unsigned long long bg = __ballot(gt), be = __ballot(eq);
        const uint32_t rg = __builtin_amdgcn_mbcnt_hi((uint32_t)(bg >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)bg, 0u));
        const uint32_t re = __builtin_amdgcn_mbcnt_hi((uint32_t)(be >> 32),
                                                      __builtin_amdgcn_mbcnt_lo((uint32_t)be, 0u));
        rk[u] = rg | (re << 8) | (gt ? 0x10000u : 0u) | (eq ? 0x20000u : 0u);
        if (lane == 0) wcnt[u * NW + w] = ((uint32_t)__popcll(bg) << 16) | (uint32_t)__popcll(be);
    }
    __syncthreads();
    // every wave scans the totals itself (exclusive, in (round, wave) order;
    // lane a holds entries 2a and 2a + 1) and takes its own entries
    const int a = 2 * lane;
    const uint32_t c0 = (a < NS) ? wcnt[a] : 0u, c1 = (a + 1 < NS) ? wcnt[a + 1] : 0u;
    const uint32_t ex = wave_prefix_sum_u32(c0 + c1) - c0 - c1;
    const int wu = __builtin_amdgcn_readfirstlane(w);
    uint32_t bf[ROUNDS];
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
        const int e = u * NW + wu;
        const uint32_t el = (uint32_t)__builtin_amdgcn_readlane((int)ex, e >> 1);
        const uint32_t cl = (uint32_t)__builtin_amdgcn_readlane((int)c0, e >> 1);
        bf[u] = el + ((e & 1) ? cl : 0u);
    }
#pragma unroll
    for (int u = 0; u < ROUNDS; ++u) {
        const int i = threadIdx.x + u * NT;
        const uint32_t g = (bf[u] >> 16) + (rk[u] & 0xffu);
        const uint32_t q = (bf[u] & 0xffffu) + ((rk[u] >> 8) & 0xffu);
        int pos = -1;
        if (rk[u] & 0x10000u) pos = (int)(g + (q < (uint32_t)need ? q : (uint32_t)need));
        else if ((rk[u] & 0x20000u) && q < (uint32_t)need) pos = (int)(g + q);
        if (pos >= 0 && pos < K) {
            okey[pos] = kv[u];
            oidx[pos] = (IDS ? iv[u] : i) + base;
        }
    }
    __syncthreads();
}

// Merge of candidate lists (each K long, ascending rows) from ckey / cidx
// into the K largest, written to okey / oidx (N = nlists * K <= PER * SEL_T
// candidates, held in registers).
template <typename V, int PER>
__device__ __forceinline__ void merge_lists_r(const uint64_t *__restrict__ ckey,
                                              const int32_t *__restrict__ cidx, int N, int K,
                                              uint64_t *okey, int32_t *oidx) {
    constexpr int SH = sizeof(V) == 8 ? 32 : 0;
    uint64_t kv[PER];
    int32_t iv[PER];
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * SEL_T;
        const uint64_t tk = ckey[i < N ? i : 0];
        const int32_t ti = cidx[i < N ? i : 0];
        kv[u] = (i < N) ? tk : 0;
        iv[u] = (i < N) ? ti : 0;
    }
    uint32_t vmx = 0u, vmn = 0xffffffffu;
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * SEL_T;
        if (i < N) {
            const uint32_t v = (uint32_t)(kv[u] >> SH);
            vmx = v > vmx ? v : vmx;
            vmn = v < vmn ? v : vmn;
        }
    }
    uint32_t vmax, vmin;
    block_minmax_u32(vmx, vmn, &vmax, &vmin);
    uint64_t T, mask;
    int need;
    radix_select<PER>(kv, N, K, SH, vmax, vmin, &T, &mask, &need);
    compact_topk<SEL_T, PER, true>(kv, iv, N, K, T, mask, need, okey, oidx, 0);
}

template <typename V>
__device__ __forceinline__ void merge_lists(const uint64_t *__restrict__ ckey,
                                            const int32_t *__restrict__ cidx, int N, int K,
                                            uint64_t *okey, int32_t *oidx) {
    if (N <= 4 * SEL_T) merge_lists_r<V, 4>(ckey, cidx, N, K, okey, oidx);
    else merge_lists_r<V, SEL_MERGE / SEL_T>(ckey, cidx, N, K, okey, oidx);
}

// The end of an iteration's selection (one workgroup): the last candidate
// merge (if do_topk and there is more than one list), the RRN from the chunk norms (strided lane sums, then a
// fixed butterfly), the stop test, the greedy set I (or the replayed one)
// with r_I, and the records.  The chunk norms are loaded together with the
// candidates.  ids / s_cn: LDS of MAXK and SEL_NCN entries.
constexpr int SEL_NCN = SEL_MERGE / 4;   // chunk norms held in LDS (the rest read again)
template <typename V>
__device__ __forceinline__ void select_final(const uint64_t *__restrict__ ckey, const int32_t *__restrict__ cidx,
                             int nlists, int K, const double *__restrict__ cn, int ncn,
                             const V *__restrict__ r, Ctrl *__restrict__ ctrl, int stop_test,
                             int do_topk, int64_t it, double *rec_rrn, int32_t *rec_I,
                             const int32_t *replay_I, int32_t *I_out, double *rI_out,
                             int32_t *ids, double *s_cn) {
    __shared__ int s_stop;
    __shared__ uint64_t fk[MAXK];
    __shared__ int32_t fi[MAXK];
    constexpr int NCN = SEL_NCN, CPT = SEL_NCN / SEL_T;
    double cnv[CPT];
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = threadIdx.x + u * SEL_T;
        cnv[u] = cn[c < ncn ? c : 0];
    }
    if (do_topk && nlists > 1) {
        merge_lists<V>(ckey, cidx, nlists * K, K, fk, fi);
        for (int p = threadIdx.x; p < K; p += SEL_T) ids[p] = fi[p];
    } else if (do_topk) {
        // one chunk: its list (ascending rows) is the top K
        for (int p = threadIdx.x; p < K; p += SEL_T) ids[p] = cidx[p];
    }
#pragma unroll
    for (int u = 0; u < CPT; ++u) {
        const int c = threadIdx.x + u * SEL_T;
        if (c < ncn) s_cn[c] = cnv[u];
    }
    __syncthreads();
    // ||r||^2 from the chunk norms: lane l of wave 0 sums chunks l, l + 64,
    // ... in order, then a fixed butterfly over the lanes
    double rn2 = 0.0;
    if (threadIdx.x < 64) {
        for (int c = threadIdx.x; c < ncn; c += 64) rn2 += (c < NCN) ? s_cn[c] : cn[c];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) rn2 += __shfl_xor(rn2, off, 64);
    }
    if (threadIdx.x == 0) {
        const double rn = sqrt(rn2);
        ctrl->rnorm2 = rn2;
        ctrl->last_it = it;
        const double bn2 = ctrl->bnorm2;
        const double rrn = (bn2 > 0.0) ? rn / sqrt(bn2) : 0.0;
        if (rec_rrn) rec_rrn[it] = rrn;
        int stop = 0;
        if (!isfinite(rn2)) {
            ctrl->status = RORBK_ERR_NONFINITE;
            stop = 1;
        } else if (stop_test && rn < ctrl->thr) {
            stop = 1;
        }
        if (stop) {
            ctrl->done = 1;
            ctrl->conv_it = it;
        }
        s_stop = stop;
    }
    __syncthreads();
    if (s_stop || !I_out) return;
    for (int p = threadIdx.x; p < K; p += SEL_T) {
        const int32_t row = replay_I ? replay_I[it * K + p] : ids[p];
        I_out[p] = row;
        rI_out[p] = (double)r[row];
        if (rec_I) rec_I[it * K + p] = row;
    }
}

// Candidate merge levels for long residuals: groups of lists_per_group lists
// (each K long) into K candidates per group; the last level (one group) ends
// the iteration's selection.
template <typename V>
__global__ __launch_bounds__(SEL_T) void k_select_merge(
    const uint64_t *__restrict__ ckey, const int32_t *__restrict__ cidx, int nlists,
    int lists_per_group, int K, uint64_t *__restrict__ okey, int32_t *__restrict__ oidx,
    int final_level, const double *__restrict__ cn, int ncn, const V *__restrict__ r,
    Ctrl *__restrict__ ctrl, int stop_test, int do_topk, int64_t it, double *rec_rrn,
    int32_t *rec_I, const int32_t *replay_I, int32_t *I_out, double *rI_out) {
    if (ctrl->done) return;
    __shared__ int32_t ids[MAXK];
    __shared__ double s_cn[SEL_NCN];
    if (final_level) {
        select_final<V>(ckey, cidx, nlists, K, cn, ncn, r, ctrl, stop_test, do_topk, it, rec_rrn,
                        rec_I, replay_I, I_out, rI_out, ids, s_cn);
        return;
    }
    const int l0 = blockIdx.x * lists_per_group;
    const int l1 = (l0 + lists_per_group < nlists) ? l0 + lists_per_group : nlists;
    merge_lists<V>(ckey + (int64_t)l0 * K, cidx + (int64_t)l0 * K, (l1 - l0) * K, K,
                   okey + (int64_t)blockIdx.x * K, oidx + (int64_t)blockIdx.x * K);
}

// What the last chunk workgroup needs to end the selection itself (fused
// form): see select_final.
template <typename V>
struct SelFinal {
    uint32_t *counter;     // NULL: not fused (a merge kernel follows)
    int nlists;
    const double *cn;
    int ncn;
    Ctrl *ctrl;
    int stop_test;
    int64_t it;
    double *rec_rrn;
    int32_t *rec_I;
    const int32_t *replay_I;
    int32_t *I_out;
    double *rI_out;
};

// LDS of the selection kernels (8-byte words): a chunk's values and block
// norms, then (fused form, last workgroup) the greedy rows and chunk norms.
constexpr int SEL_LDS = (SEL_CHUNK + SEL_BPC > MAXK / 2 + SEL_NCN) ? SEL_CHUNK + SEL_BPC
                                                                   : MAXK / 2 + SEL_NCN;
static_assert(MAXK % 2 == 0, "the chunk norms follow the greedy rows 8-byte aligned");

// The loads of a selection chunk: b and the sum over the nseg segments of the
// partial products (in segment order) for element i = threadIdx.x + u * SEL_T
// of the chunk's N rows.  FULL (every round holds rows): no branch around
// any load.  Otherwise (a short chunk, nr < PER rounds, uniform) rounds past
// the last row load nothing, since a workgroup summing many segments is
// bound by the loads it issues, and the segments go in groups of GS whose
// loads are all issued before any is added.
template <typename V, int PER, bool FULL>
__device__ __forceinline__ void chunk_loads(const V *__restrict__ b,
                                            const double *__restrict__ axp, int nseg, int64_t m,
                                            int64_t r0, int N, int nr, V (&bv)[PER],
                                            double (&av)[PER]) {
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * SEL_T;
        bv[u] = (V)0;
        if (FULL || u < nr) {
            const V t = b[r0 + (i < N ? i : 0)];
            bv[u] = (i < N) ? t : (V)0;
        }
        av[u] = 0.0;
    }
    if (!axp) return;
    int sg = 0;
    if constexpr (!FULL) {
        constexpr int GS = 4;
        for (; sg + GS <= nseg; sg += GS) {
            double t[GS][PER];
#pragma unroll
            for (int gq = 0; gq < GS; ++gq)
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int i = threadIdx.x + u * SEL_T;
                    t[gq][u] = 0.0;
                    if (u < nr) t[gq][u] = axp[(int64_t)(sg + gq) * m + r0 + (i < N ? i : 0)];
                }
#pragma unroll
            for (int gq = 0; gq < GS; ++gq)
#pragma unroll
                for (int u = 0; u < PER; ++u) {
                    const int i = threadIdx.x + u * SEL_T;
                    av[u] += (i < N) ? t[gq][u] : 0.0;
                }
        }
    }
    for (; sg < nseg; ++sg) {
        double t[PER];
#pragma unroll
        for (int u = 0; u < PER; ++u) {
            const int i = threadIdx.x + u * SEL_T;
            t[u] = 0.0;
            if (FULL || u < nr) {
                const double tv = axp[(int64_t)sg * m + r0 + (i < N ? i : 0)];
                t[u] = (i < N) ? tv : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < PER; ++u) av[u] += t[u];
    }
}

// Per selection chunk (a run of whole blocks): r_i = b_i - sum_seg axp[seg][i]
// (Algorithm 1, the full residual), per-block ||r_t||^2, the chunk's ||r||^2,
// and the chunk's local top-K candidates (keys, global row indices).  Fused
// form (fin.counter set): every workgroup publishes its results (release
// fence), counts itself done, and the last one (acquire fence) merges the
// candidates and ends the selection, so no second kernel is launched.
// SHORT: chunks with fewer rows than SEL_CHUNK take the short-chunk loads
// (the plain selection kernel; the chain form's kernel, whose chunks are
// full, keeps the one load path and its smaller register count).
template <typename V, bool SHORT>
__device__ __forceinline__ void select_chunk(
    const V *__restrict__ b, const double *__restrict__ axp, int nseg, int64_t m, int64_t q,
    int64_t rem, int64_t k, int64_t bpc, int K, V *__restrict__ r, double *__restrict__ bn,
    double *__restrict__ cn, uint64_t *__restrict__ ckey, int32_t *__restrict__ cidx,
    int do_topk, const Ctrl *__restrict__ ctrl, const SelFinal<V> &fin, int nchunks) {
    __shared__ uint64_t sel_lds[SEL_LDS];
    __shared__ int s_last;
    double *vals = reinterpret_cast<double *>(sel_lds);               // SEL_CHUNK
    double *s_bn = reinterpret_cast<double *>(sel_lds + SEL_CHUNK);   // SEL_BPC
    const int64_t t0 = (int64_t)blockIdx.x * bpc;
    const int64_t t1 = (t0 + bpc < k) ? t0 + bpc : k;
    const int64_t r0 = blk_start(t0, q, rem), r1 = blk_start(t1, q, rem);
    const int N = (int)(r1 - r0);
    constexpr int PER = SEL_CHUNK / SEL_T;
    constexpr int SH = sizeof(V) == 8 ? 32 : 0;   // the 32-bit view of a key
    // every load of the chunk in flight together with the stop flag's
    const int nr = (N + SEL_T - 1) / SEL_T;   // rounds holding rows (uniform)
    V bv[PER];
    double av[PER];
    if (!SHORT || nr == PER) chunk_loads<V, PER, true>(b, axp, nseg, m, r0, N, nr, bv, av);
    else chunk_loads<V, PER, false>(b, axp, nseg, m, r0, N, nr, bv, av);
    if (ctrl && ctrl->done) return;
    uint32_t vmx = 0u, vmn = 0xffffffffu;
    uint64_t kr[PER];   // the keys, kept in registers for the selection
#pragma unroll
    for (int u = 0; u < PER; ++u) {
        const int i = threadIdx.x + u * SEL_T;
        kr[u] = 0;
        if (i < N) {
            const V s = axp ? (V)((double)bv[u] - av[u]) : bv[u];
            const uint64_t kk = key_of(s);
            const uint32_t v = (uint32_t)(kk >> SH);
            r[r0 + i] = s;
            vals[i] = (double)s;
            kr[u] = kk;
            vmx = v > vmx ? v : vmx;
            vmn = v < vmn ? v : vmn;
        }
    }
    uint32_t vmax, vmin;
    block_minmax_u32(vmx, vmn, &vmax, &vmin);   // also orders the LDS writes above
    // per-block squared norms: 8 lanes per block, each summing every 8th row
    // in order, then a fixed butterfly over the 8 lanes
    {
        const int nb = (int)(t1 - t0), j = threadIdx.x & 7;
        for (int g = threadIdx.x >> 3; g < nb; g += SEL_T / 8) {
            const int64_t t = t0 + g;
            const int s0 = (int)(blk_start(t, q, rem) - r0);
            const int bt = blk_rows(t, q, rem);
            double s = 0.0;
#pragma unroll 4
            for (int i = j; i < bt; i += 8) s = __builtin_fma(vals[s0 + i], vals[s0 + i], s);
            s += __shfl_xor(s, 4, 64);
            s += __shfl_xor(s, 2, 64);
            s += __shfl_xor(s, 1, 64);
            if (j == 0) {
                bn[t] = s;
                s_bn[g] = s;
            }
        }
    }
    __syncthreads();
    // the chunk's ||r||^2: wave 0, lane l summing blocks l, l + 64, ... in
    // order, then a fixed butterfly over the lanes
    if (threadIdx.x < 64) {
        const int nb = (int)(t1 - t0);
        double s = 0.0;
        for (int g = threadIdx.x; g < nb; g += 64) s += s_bn[g];
#pragma unroll
        for (int off = 32; off >= 1; off >>= 1) s += __shfl_xor(s, off, 64);
        if (threadIdx.x == 0) cn[blockIdx.x] = s;
    }
    if (do_topk) {
        uint64_t T, mask;
        int need;
        const int32_t none[PER] = {};   // (positions stand for the indices)
        radix_select<PER>(kr, N, K, SH, vmax, vmin, &T, &mask, &need);
        compact_topk<SEL_T, PER, false>(kr, none, N, K, T, mask, need,
                                        ckey + (int64_t)blockIdx.x * K,
                                        cidx + (int64_t)blockIdx.x * K, (int32_t)r0);
    }
    if (!fin.counter) return;
    // count this workgroup done; the acquire-release device-scope atomic
    // publishes its r, norms and candidates and, for the last one, makes
    // every other workgroup's visible
    __syncthreads();
    if (threadIdx.x == 0)
        s_last = (__hip_atomic_fetch_add(fin.counter, 1u, __ATOMIC_ACQ_REL,
                                         __HIP_MEMORY_SCOPE_AGENT) == (uint32_t)nchunks - 1) ? 1 : 0;
    __syncthreads();
    if (!s_last) return;
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    if (threadIdx.x == 0) *fin.counter = 0u;   // ready for the next launch
    select_final<V>(ckey, cidx, fin.nlists, K, fin.cn, fin.ncn, r, fin.ctrl, fin.stop_test,
                    do_topk, fin.it, fin.rec_rrn, fin.rec_I, fin.replay_I, fin.I_out, fin.rI_out,
                    reinterpret_cast<int32_t *>(sel_lds),
                    reinterpret_cast<double *>(sel_lds + MAXK / 2));
}

template <typename V>
__global__ __launch_bounds__(SEL_T) void k_select_chunk(
    const V *__restrict__ b, const double *__restrict__ axp, int nseg, int64_t m, int64_t q,
    int64_t rem, int64_t k, int64_t bpc, int K, V *__restrict__ r, double *__restrict__ bn,
    double *__restrict__ cn, uint64_t *__restrict__ ckey, int32_t *__restrict__ cidx,
    int do_topk, const Ctrl *__restrict__ ctrl, SelFinal<V> fin) {
    select_chunk<V, true>(b, axp, nseg, m, q, rem, k, bpc, K, r, bn, cn, ckey, cidx, do_topk, ctrl,
                          fin, (int)gridDim.x);
}

// The cross-Grams of the next iteration's blocks (xgram_tile with one wave
// per 64 of the SEL_T threads) in spare workgroups after the nchunks selection
// chunks: they need no result of this iteration, and the selection's few
// workgroups leave the rest of the chip idle.
struct XgSel {
    const void *A;
    int64_t ld, n, q, rem;
    int bmax;
    const int32_t *tau;
    int64_t ti;
    double *out;
};

template <typename V, typename T, bool AL>
__global__ __launch_bounds__(SEL_T) void k_select_xg(
    const V *__restrict__ b, const double *__restrict__ axp, int nseg, int64_t m, int64_t q,
    int64_t rem, int64_t k, int64_t bpc, int K, V *__restrict__ r, double *__restrict__ bn,
    double *__restrict__ cn, uint64_t *__restrict__ ckey, int32_t *__restrict__ cidx,
    int do_topk, const Ctrl *__restrict__ ctrl, SelFinal<V> fin, int nchunks, XgSel xs) {
    if ((int)blockIdx.x >= nchunks) {
        xgram_tile<T, AL, SEL_T / 64>((const T *)xs.A, xs.ld, xs.n, xs.tau, xs.ti, xs.q, xs.rem,
                                      xs.bmax, (int)blockIdx.x - nchunks, xs.out);
        return;
    }
    select_chunk<V, false>(b, axp, nseg, m, q, rem, k, bpc, K, r, bn, cn, ckey, cidx, do_topk, ctrl,
                           fin, nchunks);
}
static_assert(SEL_T == 512, "the selection's spare workgroups run the 8-wave cross-Gram tiles");


hipError_t launch_select(const rorbk_handle_s *h, const SelectArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    const int K = (int)L.K;
    const int do_topk = (!a.skip_topk && !a.replay_I) ? 1 : 0;
    // one merge of all chunk candidates fits a workgroup: fuse it into the
    // chunk kernel (its last workgroup); otherwise merge in levels
    const int per = SEL_MERGE / K;
    const bool fuse = !do_topk || L.nch_s <= per;
#define RORBK_SEL(V)                                                                            \
    do {                                                                                        \
        SelFinal<V> fin = {};                                                                   \
        if (fuse) {                                                                             \
            fin.counter = h->d_selcnt;                                                          \
            fin.nlists = L.nch_s;                                                               \
            fin.cn = h->d_cn;                                                                   \
            fin.ncn = L.nch_s;                                                                  \
            fin.ctrl = h->d_ctrl;                                                               \
            fin.stop_test = a.stop_test;                                                        \
            fin.it = a.it;                                                                      \
            fin.rec_rrn = a.record_rrn ? a.rec_rrn : nullptr;                                   \
            fin.rec_I = a.record_I ? a.rec_I : nullptr;                                         \
            fin.replay_I = a.replay_I;                                                          \
            fin.I_out = a.I_out;                                                                \
            fin.rI_out = a.rI_out;                                                              \
        }                                                                                       \
        if (a.xg_out && fuse) {                                                                 \
            XgSel xs = {a.xg_A, L.ld, L.n, L.q, L.rem, (int)L.bmax, h->d_tau, a.xg_ti, a.xg_out};  \
            const int nx = xgram_jobs((int)L.bmax);                                             \
            RORBK_SEL_XG(V, double, RORBK_F64);                                                 \
            RORBK_SEL_XG(V, float, RORBK_F32);                                                  \
            RORBK_SEL_XG(V, bf16_t, RORBK_BF16);                                                \
            (void)nx;                                                                           \
        } else {                                                                                \
            hipLaunchKernelGGL(k_select_chunk<V>, dim3(L.nch_s), dim3(SEL_T), 0, s,             \
                               (const V *)a.b, a.axp, a.nseg, L.m, L.q, L.rem, L.k, L.bpc, K,   \
                               (V *)a.r, h->d_bn, h->d_cn, h->d_ckey, h->d_cidx, do_topk,       \
                               h->d_ctrl, fin);                                                 \
        }                                                                                       \
    } while (0)
#define RORBK_SEL_XG(V, T, DT)                                                                  \
    if (a.xg_dt == DT) {                                                                        \
        if (a.xg_aligned)                                                                       \
            hipLaunchKernelGGL((k_select_xg<V, T, true>), dim3(L.nch_s + nx), dim3(SEL_T), 0, s, \
                               (const V *)a.b, a.axp, a.nseg, L.m, L.q, L.rem, L.k, L.bpc, K,   \
                               (V *)a.r, h->d_bn, h->d_cn, h->d_ckey, h->d_cidx, do_topk,       \
                               h->d_ctrl, fin, (int)L.nch_s, xs);                               \
        else                                                                                    \
            hipLaunchKernelGGL((k_select_xg<V, T, false>), dim3(L.nch_s + nx), dim3(SEL_T), 0,  \
                               s, (const V *)a.b, a.axp, a.nseg, L.m, L.q, L.rem, L.k, L.bpc,   \
                               K, (V *)a.r, h->d_bn, h->d_cn, h->d_ckey, h->d_cidx, do_topk,    \
                               h->d_ctrl, fin, (int)L.nch_s, xs);                               \
    }
    if (a.xg_out && !fuse) return hipErrorInvalidValue;   // the chain form needs one level
    if (a.vec == VEC_F64) RORBK_SEL(double);
    else RORBK_SEL(float);
#undef RORBK_SEL
#undef RORBK_SEL_XG
    hipError_t e = hipGetLastError();
    if (e != hipSuccess || fuse) return e;
    // merge levels: lists of K candidates, at most SEL_MERGE per workgroup
    int nlists = L.nch_s;
    const uint64_t *ik = h->d_ckey;
    const int32_t *ii = h->d_cidx;
    int flip = 0;
    while (nlists > per) {
        const int groups = (nlists + per - 1) / per;
        uint64_t *ok = flip ? h->d_ckey : h->d_ckey2;
        int32_t *oi = flip ? h->d_cidx : h->d_cidx2;
        if (a.vec == VEC_F64)
            hipLaunchKernelGGL(k_select_merge<double>, dim3(groups), dim3(SEL_T), 0, s, ik, ii,
                               nlists, per, K, ok, oi, 0, nullptr, 0, (const double *)nullptr,
                               h->d_ctrl, 0, 1, a.it, nullptr, nullptr, nullptr, nullptr, nullptr);
        else
            hipLaunchKernelGGL(k_select_merge<float>, dim3(groups), dim3(SEL_T), 0, s, ik, ii,
                               nlists, per, K, ok, oi, 0, nullptr, 0, (const float *)nullptr,
                               h->d_ctrl, 0, 1, a.it, nullptr, nullptr, nullptr, nullptr, nullptr);
        e = hipGetLastError();
        if (e != hipSuccess) return e;
        ik = ok;
        ii = oi;
        nlists = groups;
        flip ^= 1;
    }
    if (a.vec == VEC_F64)
        hipLaunchKernelGGL(k_select_merge<double>, dim3(1), dim3(SEL_T), 0, s, ik, ii, nlists,
                           nlists, K, nullptr, nullptr, 1, h->d_cn, L.nch_s, (const double *)a.r,
                           h->d_ctrl, a.stop_test, do_topk, a.it,
                           a.record_rrn ? a.rec_rrn : nullptr, a.record_I ? a.rec_I : nullptr,
                           a.replay_I, a.I_out, a.rI_out);
    else
        hipLaunchKernelGGL(k_select_merge<float>, dim3(1), dim3(SEL_T), 0, s, ik, ii, nlists,
                           nlists, K, nullptr, nullptr, 1, h->d_cn, L.nch_s, (const float *)a.r,
                           h->d_ctrl, a.stop_test, do_topk, a.it,
                           a.record_rrn ? a.rec_rrn : nullptr, a.record_I ? a.rec_I : nullptr,
                           a.replay_I, a.I_out, a.rI_out);
    return hipGetLastError();
}

// ------------------------------------------------------ greedy block solve --
// (A_I A_I^T + lambda I) y = rhs, the greedy step of Algorithm 1, rhs = r_I
// (forward) or, for the adjoint, -(sum of the partial products A_I g).  Greedy
// sets of at most 64 rows are solved by k_chol_wave below; larger ones by the
// blocked Cholesky on 32 x 32 tiles (one launch per tile column, k_big.hip).
// A pivot that is not positive (or not finite) sets RORBK_ERR_NOT_SPD.

// Packed Gram partials summed in chunk order into LDS, KP <= NU * 256: thread
// t owns elements t + 256 u (u < NU) and keeps CG chunks of each in flight
// together (about 72 loads).  Addresses are clamped into the buffer and the
// extra values scaled by zero, so no load sits behind a branch.
template <int NU>
__device__ __forceinline__ void gram_sum_chunks(const double *__restrict__ Gpart, int nch, int KP,
                                                double *__restrict__ Gp) {
    constexpr int NTH = 256, CG = 8 * (9 / NU);
    double g[NU];
#pragma unroll
    for (int u = 0; u < NU; ++u) g[u] = 0.0;
    for (int c0 = 0; c0 < nch; c0 += CG) {
        double t[NU][CG];
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int c = 0; c < CG; ++c) {
                const int f = threadIdx.x + u * NTH;
                const int fc = (f < KP) ? f : KP - 1;
                const int cc = (c0 + c < nch) ? c0 + c : nch - 1;
                const double keep = (f < KP && c0 + c < nch) ? 1.0 : 0.0;
                t[u][c] = Gpart[(int64_t)cc * KP + fc] * keep;
            }
#pragma unroll
        for (int u = 0; u < NU; ++u)
#pragma unroll
            for (int c = 0; c < CG; ++c) g[u] += t[u][c];
    }
#pragma unroll
    for (int u = 0; u < NU; ++u) {
        const int f = threadIdx.x + u * NTH;
        if (f < KP) Gp[f] = g[u];
    }
}

// K <= 64: the whole solve on one wave (panel LDL^T with MFMA updates, ldl_blk64).
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(1, 1))) void k_chol_wave(
    const double *__restrict__ Gpart, int nch, int K, double lambda,
    const double *__restrict__ rI, const double *__restrict__ Pin, int nchP, int bmax,
    double *__restrict__ y, Ctrl *__restrict__ ctrl) {
    constexpr int NTH = 256;
    __shared__ double Gp[64 * 65 / 2];
    __shared__ double z[64];
    __shared__ double colbuf[2 * 64];
    __shared__ double Lc[64 * 65];
    // the stop flag is read by a vector load issued with the chunk loads (the
    // Gram buffer is valid either way), so the two latencies overlap
    const int stop = __hip_atomic_load(&ctrl->done, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const int KP = K * (K + 1) / 2;
    // NU packed elements per thread, CG chunks of each in flight together
    switch ((KP + NTH - 1) / NTH) {
        case 1: gram_sum_chunks<1>(Gpart, nch, KP, Gp); break;
        case 2: gram_sum_chunks<2>(Gpart, nch, KP, Gp); break;
        case 3: gram_sum_chunks<3>(Gpart, nch, KP, Gp); break;
        case 4: gram_sum_chunks<4>(Gpart, nch, KP, Gp); break;
        case 5: gram_sum_chunks<5>(Gpart, nch, KP, Gp); break;
        case 6: gram_sum_chunks<6>(Gpart, nch, KP, Gp); break;
        case 7: gram_sum_chunks<7>(Gpart, nch, KP, Gp); break;
        case 8: gram_sum_chunks<8>(Gpart, nch, KP, Gp); break;
        default: gram_sum_chunks<9>(Gpart, nch, KP, Gp); break;
    }
    if (stop) return;
    for (int q = threadIdx.x; q < K; q += NTH) {
        if (rI) {
            z[q] = rI[q];
        } else {
            double sacc = 0.0;
            for (int c = 0; c < nchP; ++c) sacc += Pin[(int64_t)c * bmax + q];
            z[q] = -sacc;
        }
    }
    __syncthreads();
    // the padded system (lambda on the diagonal, the identity beyond K)
    for (int f = threadIdx.x; f < 64 * 65 / 2; f += NTH) lb_put(Lc, f, (f < KP) ? Gp[f] : 0.0, K, lambda);
    for (int q = K + (int)threadIdx.x; q < 64; q += NTH) z[q] = 0.0;
    __syncthreads();
    // one wave from here on; the other waves leave and no block barrier follows
    if (threadIdx.x >= 64) return;
    if (!ldl_blk64(Lc, z, K, colbuf)) {
        if (threadIdx.x == 0) {
            ctrl->status = RORBK_ERR_NOT_SPD;
            ctrl->done = 1;
        }
        return;
    }
    for (int q = threadIdx.x; q < K; q += 64) y[q] = z[q];
}

hipError_t launch_chol_solve(const rorbk_handle_s *h, const double *Gpart, int K,
                             const double *rI, const double *Pin, double *y, hipStream_t s) {
    const Layout &L = h->L;
    if (K > 64) {
        // the handle holds the blocked factorisation's buffers for every
        // greedy set of more than 64 rows
        if (!h->d_bigG) return hipErrorInvalidValue;
        return launch_big_chol_solve(h, Gpart, K, rI, Pin, y, s);
    }
    hipLaunchKernelGGL(k_chol_wave, dim3(1), dim3(256), 0, s, Gpart, L.nch_g, K, h->lambda, rI,
                       Pin, L.nch_u, (int)L.bmax, y, h->d_ctrl);
    return hipGetLastError();
}

// ------------------------------------------------------ initial solution --
// Algorithm 2 (appendix): y = the sum of the rows of A, kept from the setup as
// the sum of the block row-sums (centroids).  A workgroup takes 64 columns;
// wave w sums the blocks of its contiguous sixteenth in block order (one
// coalesced 64-column read per block, eight in flight), and wave 0 adds the
// sixteen partial sums in wave order.
__global__ __launch_bounds__(1024) void k_colsum(const double *__restrict__ cen, int64_t k,
                                                 int64_t n, double *__restrict__ y) {
    __shared__ double part[16][64];
    constexpr int U = 8;
    const int lane = threadIdx.x & 63, w = threadIdx.x >> 6;
    const int64_t j = (int64_t)blockIdx.x * 64 + lane;
    const int64_t per = (k + 15) / 16;
    const int64_t t0 = w * per, t1 = (t0 + per < k) ? t0 + per : k;
    const int64_t jc = (j < n) ? j : n - 1;
    double s = 0.0;
    int64_t t = t0;
    for (; t + U <= t1; t += U) {
        double v[U];
#pragma unroll
        for (int u = 0; u < U; ++u) v[u] = cen[(t + u) * n + jc];
#pragma unroll
        for (int u = 0; u < U; ++u) s += v[u];
    }
    for (; t < t1; ++t) s += cen[t * n + jc];
    part[w][lane] = s;
    __syncthreads();
    if (w == 0 && j < n) {
        double a = part[0][lane];
        for (int v2 = 1; v2 < 16; ++v2) a += part[v2][lane];
        y[j] = a;
    }
}

// The coefficient <b, b~> / ||b~||^2 of Algorithm 2 with b~ = A y given as the
// residual pass's segment products (summed in segment order): thread t sums
// rows t, t + 1024, ... in order, then a fixed-order workgroup sum.
// out[0] = <b, b~>, out[1] = ||b~||^2, out[2] = the coefficient (0 if b~ = 0).
template <typename V>
__global__ __launch_bounds__(1024) void k_alg2_coef(const V *__restrict__ b,
                                                    const double *__restrict__ axp, int nseg,
                                                    int64_t m, double *__restrict__ out) {
    __shared__ double sh[16];
    double sb = 0.0, st = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += blockDim.x) {   // coalesced, rows in order per thread
        double bt = 0.0;
        for (int sg = 0; sg < nseg; ++sg) bt += axp[(int64_t)sg * m + i];
        sb = __builtin_fma((double)b[i], bt, sb);
        st = __builtin_fma(bt, bt, st);
    }
    sb = block_sum(sb, sh);
    st = block_sum(st, sh);
    if (threadIdx.x == 0) {
        out[0] = sb;
        out[1] = st;
        out[2] = (st > 0.0) ? sb / st : 0.0;
    }
}

template <typename V>
__global__ __launch_bounds__(256) void k_scale_vec(const double *__restrict__ y,
                                                   const double *__restrict__ coef,
                                                   V *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] = (V)(coef[0] * y[i]);
}

hipError_t launch_colsum(const double *cen, int64_t k, int64_t n, double *y, hipStream_t s) {
    hipLaunchKernelGGL(k_colsum, dim3((unsigned)((n + 63) / 64)), dim3(1024), 0, s, cen, k, n, y);
    return hipGetLastError();
}

hipError_t launch_alg2(const void *b, int vec, const double *axp, int nseg, int64_t m,
                       const double *y, double *coef, void *x, int64_t n, hipStream_t s) {
    const unsigned g = (unsigned)((n + 255) / 256);
    if (vec == VEC_F64) {
        hipLaunchKernelGGL(k_alg2_coef<double>, dim3(1), dim3(1024), 0, s, (const double *)b, axp,
                           nseg, m, coef);
        hipLaunchKernelGGL(k_scale_vec<double>, dim3(g), dim3(256), 0, s, y, coef + 2,
                           (double *)x, n);
    } else {
        hipLaunchKernelGGL(k_alg2_coef<float>, dim3(1), dim3(1024), 0, s, (const float *)b, axp,
                           nseg, m, coef);
        hipLaunchKernelGGL(k_scale_vec<float>, dim3(g), dim3(256), 0, s, y, coef + 2,
                           (float *)x, n);
    }
    return hipGetLastError();
}

// -------------------------------------------------------- refinement glue --
__global__ void k_cast_f64_f32(const double *__restrict__ a, float *__restrict__ b, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) b[i] = (float)a[i];
}
__global__ void k_axpy_f32_f64(const float *__restrict__ d, double *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += (double)d[i];
}
__global__ void k_zero(uint32_t *p, int64_t words) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < words) p[i] = 0u;
}

hipError_t launch_cast_f64_to_f32(const double *src, float *dst, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_cast_f64_f32, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, src,
                       dst, n);
    return hipGetLastError();
}
hipError_t launch_axpy_f32_to_f64(const float *d, double *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_f32_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, x,
                       n);
    return hipGetLastError();
}
hipError_t launch_fill_zero(void *p, int64_t bytes, hipStream_t s) {
    const int64_t words = bytes / 4;
    if (words <= 0) return hipSuccess;
    hipLaunchKernelGGL(k_zero, dim3((unsigned)((words + 255) / 256)), dim3(256), 0, s,
                       (uint32_t *)p, words);
    return hipGetLastError();
}

// Inner stop threshold of a refinement step: the inner residual estimates
// b - A(x + d); stop once it is below max(eta ||r_out||, tol ||b||).  The
// recorded RRN stays relative to the original ||b||.
__global__ void k_refine_ctrl(Ctrl *c, double tol, double eta, const double *__restrict__ rout2,
                              double bnorm2) {
    c->done = 0;
    c->status = 0;
    c->bnorm2 = bnorm2;
    const double a = eta * sqrt(*rout2), bb = tol * sqrt(bnorm2);
    c->thr = a > bb ? a : bb;
}

__global__ void k_init_ctrl(Ctrl *c, double tol, const double *__restrict__ bnorm2) {
    c->done = 0;
    c->status = 0;
    c->conv_it = -1;
    c->bnorm2 = *bnorm2;
    c->thr = tol * sqrt(*bnorm2);
    c->rnorm2 = 0.0;
    c->last_it = -1;
}

hipError_t launch_init_ctrl(Ctrl *c, double tol, const double *bnorm2, hipStream_t s) {
    hipLaunchKernelGGL(k_init_ctrl, dim3(1), dim3(1), 0, s, c, tol, bnorm2);
    return hipGetLastError();
}

__global__ void k_set_thr(Ctrl *c, double thr) { c->thr = thr; }

hipError_t launch_set_thr(Ctrl *c, double thr, hipStream_t s) {
    hipLaunchKernelGGL(k_set_thr, dim3(1), dim3(1), 0, s, c, thr);
    return hipGetLastError();
}

__global__ void k_axpy_f64(const double *__restrict__ d, double *__restrict__ x, int64_t n) {
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i < n) x[i] += d[i];
}

hipError_t launch_axpy_f64(const double *d, double *x, int64_t n, hipStream_t s) {
    hipLaunchKernelGGL(k_axpy_f64, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, d, x, n);
    return hipGetLastError();
}

hipError_t launch_set_refine_ctrl(Ctrl *c, double tol, double eta, const double *rout2,
                                  double outer_bnorm2, hipStream_t s) {
    hipLaunchKernelGGL(k_refine_ctrl, dim3(1), dim3(1), 0, s, c, tol, eta, rout2, outer_bnorm2);
    return hipGetLastError();
}

}  // namespace rorbk
