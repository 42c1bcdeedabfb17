// k_big.hip -- ROR-BK with blocks of more than MAXB rows (up to BIGB) on a
// dense matrix: the regime of the paper's own experiments, which split A into
// 100 blocks (Section 3.1, Tables 3 and 5), i.e. hundreds of rows per block.
// Such a block fits neither a workgroup's registers nor its LDS, so the work of
// one step is spread over the chip:
//  - the symmetric positive definite systems (each fixed block's Gram at setup,
//    the greedy block's Gram every iteration) are factored by a right-looking
//    blocked Cholesky on 32 x 32 tiles in global memory, batched over
//    matrices, one launch per tile column: every workgroup scales the two
//    panel tiles it needs by the inverse of the diagonal tile and updates one
//    trailing tile (FP64 MFMA), and the workgroup of the next diagonal tile
//    factors and inverts it at once.  Matrices are padded to whole tiles with
//    the identity.  The greedy system carries its right-hand side as an extra
//    tile row, so the factorisation also performs the forward solve;
//  - the setup then forms L^{-1} by tile rows and the stored inverse
//    H_t = L^{-T} L^{-1}, exactly symmetric;
//  - a fixed block step is four kernels: r_S from the partial products, y =
//    H_t r_S, the update's column partial sums over row chunks, and the
//    application x += sum of the partials fused with the next rows' partial
//    products.  A greedy step replaces the first two by the factorisation and
//    a backward solve.
// Every sum is taken in a fixed order, so results are reproducible.
#include "rorbk_device.h"
#include "gram_tiles.h"

namespace rorbk {

constexpr int TB = 32;        // tile size of the blocked factorisation
constexpr int BIG_T = 512;    // threads of the update kernels
constexpr int BIG_RPT = 8;    // rows per thread in the update kernels

// Rows per chunk of the update kernels for storage T: row groups x BIG_RPT
// (64 for FP64, 128 for FP32, 256 for BF16).
template <typename T>
constexpr int big_rch() { return (BIG_T / (128 / Tr<T>::VW)) * BIG_RPT; }

__device__ __forceinline__ bool ctrl_done(const Ctrl *c) { return c && c->done; }

// ------------------------------------------------------------ Cholesky ----
// Padded matrices G[bt] of `rows` x ld (row-major, ld = P * TB, rows = ld or
// ld + TB with the right-hand-side tile row) from packed lower sums:
// element (i, j) = sum_{c < nsum} src[bt * mstride + c * cstride + pk(i, j)]
// (+ lambda on the diagonal) for i, j < K; the identity past K; zero above the
// diagonal.  Row ld (greedy form) holds the right-hand side: rI, or for the
// adjoint -(sum over nchP partial products Pin[c * bmax + j]).
// Matrix bt of the batch is block t0 + bt (fixedK = 0) or has size fixedK.
__global__ __launch_bounds__(256) void k_big_unpack(const double *__restrict__ src,
                                                    int64_t mstride, int64_t cstride, int nsum,
                                                    int fixedK, int64_t t0, int64_t q, int64_t rem,
                                                    double lambda, int ld, int rows,
                                                    const double *__restrict__ rI,
                                                    const double *__restrict__ Pin, int nchP,
                                                    int bmax, double *__restrict__ G,
                                                    const Ctrl *__restrict__ ctrl) {
    if (ctrl_done(ctrl)) return;
    const int bt = blockIdx.y;
    const int K = fixedK > 0 ? fixedK : blk_rows(t0 + bt, q, rem);
    const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (e >= (int64_t)rows * ld) return;
    const int i = (int)(e / ld), j = (int)(e % ld);
    double v = 0.0;
    if (i < ld) {
        if (j <= i) {
            if (i < K) {
                const double *s = src + (int64_t)bt * mstride + pk(i, j);
                for (int c = 0; c < nsum; ++c) v += s[(int64_t)c * cstride];
                if (i == j) v += lambda;
            } else {
                v = (i == j) ? 1.0 : 0.0;
            }
        }
    } else if (i == ld && j < K) {
        if (rI) {
            v = rI[j];
        } else {
            double s = 0.0;
            for (int c = 0; c < nchP; ++c) s += Pin[(int64_t)c * bmax + j];
            v = -s;
        }
    }
    G[(int64_t)bt * rows * ld + e] = v;
}

// Orders one wave's LDS accesses across lanes (a compiler barrier for memory
// operations; LDS instructions of one wave execute in order).
__device__ __forceinline__ void wsync() {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    __builtin_amdgcn_wave_barrier();
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / sqrt(d): the hardware estimate refined by two steps of Newton's
// iteration for the reciprocal square root, r <- r (3 - d r^2) / 2.
__device__ __forceinline__ double rsq_nr(double d) {
    double r = __builtin_amdgcn_rsq(d);
#pragma unroll
    for (int it = 0; it < 2; ++it) {
        const double h = d * r;
        const double e = __builtin_fma(-h, r, 1.0);
        r = __builtin_fma(0.5 * r, e, r);
    }
    return r;
}

// 16 x 16 MFMA product on one wave from LDS (row strides RA, RB):
// acc += A B^T (TRANSB) or A B.  Result element (i, j) sits in register i / 4
// of lane (i % 4) * 16 + j; k is summed in steps of 4, in order.
template <bool TRANSB>
__device__ __forceinline__ dvec4 mm16(const double *A, int RA, const double *B, int RB, dvec4 acc) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int k0 = 0; k0 < 16; k0 += 4) {
        const double a = A[li * RA + k0 + lk];
        const double b = TRANSB ? B[li * RB + k0 + lk] : B[(k0 + lk) * RB + li];
        acc = __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, acc, 0, 0, 0);
    }
    return acc;
}

__device__ __forceinline__ void st16(double *D, int RD, dvec4 v, double scale) {
    const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
    for (int r = 0; r < 4; ++r) D[(lk + 4 * r) * RD + li] = scale * v[r];
}

// Broadcast of lane J of each 16-lane row to the whole row (DPP row_newbcast,
// one 64-bit move, the value stays in vector registers).
template <int J>
__device__ __forceinline__ double rowbc(double v) {
    return __builtin_amdgcn_mov_dpp(v, 0x150 + J, 0xf, 0xf, false);
}

// Pieces of one elimination step of f16 (compile-time indices, so every
// register index is static): the trailing update of row i of the block and
// the update of row i of the running transformation.
// acc += (src of lane J of the 16-lane row) * mul.
template <int J>
__device__ __forceinline__ void fmac_bc(double &acc, double src, double mul) {
    acc = __builtin_fma(rowbc<J>(src), mul, acc);
}

template <int k, int J>
__device__ __forceinline__ void f16_a1(double (&a)[16], double nl, double akk) {
    if constexpr (J > k) fmac_bc<J>(a[J], akk, nl);
}
template <int k, int J>
__device__ __forceinline__ void f16_e1(double (&e)[16], double nle) {
    if constexpr (J <= k) fmac_bc<k>(e[J], e[J], nle);
}

// Elimination step k of the LDL^T factorisation (unit lower factor U, pivots
// d_k).  Lane i holds row i of the block (a) and row i of the running
// transformation T (e, from the identity).  With u_ik = a_ik / d_k: rows
// i > k take a_ij -= u_ik a_jk (j > k) and e_ij -= u_ik e_kj (j <= k); u_ik is
// kept in a_ik.  1 / d_k is the hardware reciprocal r0 refined by Newton's
// iteration, r1 = r0 (2 - d r0) and r2 = r1 (2 - d r1), with the last step
// folded into its uses (u = a r1 + a r1 (1 - d r1)).  The next pivot is formed
// straight from this one, d_{k+1} = a_{k+1,k+1} - a_{k+1,k}^2 / d_k, so the
// chain from pivot to pivot is a few dependent operations; the broadcasts of
// the a_jk do not wait for it.  After the last step a holds U below the
// diagonal and e holds U^{-1}; `down` holds the lane's own pivot.
template <int k, int... J>
__device__ __forceinline__ void f16_step(double (&a)[16], double (&e)[16], double &down,
                                         double &dnext, int i, bool &ok,
                                         std::integer_sequence<int, J...>) {
    const double d = rowbc<k>(dnext);
    ok = ok && (d > 0.0) && isfinite(d);
    const double r0 = __builtin_amdgcn_rcp(d);
    const double e0 = __builtin_fma(-d, r0, 1.0);
    const double r1 = __builtin_fma(r0, e0, r0);
    const double e1 = __builtin_fma(-d, r1, 1.0);
    const double akk = a[k];
    const double m1 = akk * r1;
    const double l = __builtin_fma(m1, e1, m1);
    if constexpr (k + 1 < 16) {
        const double t = akk * akk;
        const double tr1 = t * r1;
        const double u = __builtin_fma(-t, r1, a[k + 1]);
        dnext = __builtin_fma(-tr1, e1, u);
    }
    (f16_a1<k, J>(a, -l, akk), ...);
    const double nle = (i > k) ? -l : 0.0;   // transformation rows below the pivot only
    (f16_e1<k, J>(e, nle), ...);
    a[k] = (i == k) ? akk : l;
    down = (i == k) ? d : down;
}

template <int J>
__device__ __forceinline__ void f16_scale1(double (&a)[16], double sq) {
    a[J] *= rowbc<J>(sq);
}

template <int... K>
__device__ __forceinline__ void f16_steps(double (&a)[16], double (&e)[16], double &down, int i,
                                          bool &ok, std::integer_sequence<int, K...>) {
    double dnext = a[0];
    (f16_step<K>(a, e, down, dnext, i, ok, std::make_integer_sequence<int, 16>{}), ...);
}

template <int... J>
__device__ __forceinline__ void f16_scale(double (&a)[16], double sq,
                                          std::integer_sequence<int, J...>) {
    (f16_scale1<J>(a, sq), ...);
}

// Cholesky factor and inverse of a 16 x 16 SPD block in LDS (row stride RS) on
// one wave, lane i & 15 holding row i (every 16-lane row of the wave carries
// the same copy), from the LDL^T elimination: L = U D^{1/2} and L^{-1} =
// D^{-1/2} U^{-1}, with 1 / sqrt(d_i) from rsq_nr.  The block is overwritten
// by L (zeros above the diagonal) and Wl receives L^{-1}.
__device__ __forceinline__ void f16(double *S, int RS, double *Wl, bool &ok) {
    const int lane = threadIdx.x & 63, i = lane & 15;
    double a[16], e[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
        a[j] = (j <= i) ? S[i * RS + j] : 0.0;
        e[j] = (j == i) ? 1.0 : 0.0;
    }
    double down = 1.0;
    f16_steps(a, e, down, i, ok, std::make_integer_sequence<int, 16>{});
    const double s = rsq_nr(down), sq = down * s;   // 1 / sqrt(d_i), sqrt(d_i)
    f16_scale(a, sq, std::make_integer_sequence<int, 16>{});   // u_ij sqrt(d_j)
    wsync();
    if (lane < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) {
            S[i * RS + j] = (j < i) ? a[j] : ((j == i) ? sq : 0.0);
            Wl[i * RS + j] = (j <= i) ? e[j] * s : 0.0;
        }
    }
    wsync();
}

// Cholesky factor L and inverse W = L^{-1} of a 32 x 32 SPD tile in LDS (lower
// part read; overwritten by L with zeros above), in two levels of 16:
// L11, W11; L21 = A21 W11^T; A22 -= L21 L21^T; L22, W22; W21 = -W22 L21 W11.
// Runs on wave 0; ends with a workgroup barrier.  Returns false (to wave 0) if
// a pivot is not positive.
__device__ bool tile_factor32(double (*S)[TB + 1], double (*Wl)[TB + 1]) {
    bool ok = true;
    if (threadIdx.x < 64) {
        constexpr int RS = TB + 1;
        const dvec4 z4 = {0.0, 0.0, 0.0, 0.0};
        f16(&S[0][0], RS, &Wl[0][0], ok);
        const dvec4 l21 = mm16<true>(&S[16][0], RS, &Wl[0][0], RS, z4);
        wsync();
        st16(&S[16][0], RS, l21, 1.0);
        wsync();
        const dvec4 u = mm16<true>(&S[16][0], RS, &S[16][0], RS, z4);
        {
            const int l = threadIdx.x & 63, li = l & 15, lk = l >> 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) S[16 + lk + 4 * r][16 + li] -= u[r];
        }
        wsync();
        f16(&S[16][16], RS, &Wl[16][16], ok);
        const dvec4 t1 = mm16<false>(&S[16][0], RS, &Wl[0][0], RS, z4);     // L21 W11
        wsync();
        st16(&Wl[16][0], RS, t1, 1.0);
        wsync();
        const dvec4 w21 = mm16<false>(&Wl[16][16], RS, &Wl[16][0], RS, z4);  // W22 (L21 W11)
        wsync();
        st16(&Wl[16][0], RS, w21, -1.0);
        {
            const int l = threadIdx.x & 63;
            for (int e = l; e < 256; e += 64) {
                S[e >> 4][16 + (e & 15)] = 0.0;
                Wl[e >> 4][16 + (e & 15)] = 0.0;
            }
        }
        wsync();
    }
    __syncthreads();
    return ok;
}

// 32 x 32 products on four waves from LDS: wave w computes the 16 x 16
// sub-tile (w / 2, w % 2) of A B^T; k summed in order.
__device__ __forceinline__ dvec4 mm32_abt(const double (*A)[TB + 1], const double (*B)[TB + 1]) {
    const int w = threadIdx.x >> 6, R = w >> 1, C = w & 1;
    const dvec4 z4 = {0.0, 0.0, 0.0, 0.0};
    dvec4 acc = mm16<true>(&A[R * 16][0], TB + 1, &B[C * 16][0], TB + 1, z4);
    return mm16<true>(&A[R * 16][16], TB + 1, &B[C * 16][16], TB + 1, acc);
}

__device__ __forceinline__ void st32(double (*D)[TB + 1], dvec4 v) {
    const int w = threadIdx.x >> 6, R = w >> 1, C = w & 1;
    st16(&D[R * 16][C * 16], TB + 1, v, 1.0);
}

// 32 x 32 tiles on 256 threads: thread t takes entries t + 256 u (u < 4); the
// four loads of a tile are issued before any of them is stored to LDS.
constexpr int TU = TB * TB / 256;

__device__ __forceinline__ void tile_fetch(const double *src, int ld, double (&v)[TU]) {
#pragma unroll
    for (int u = 0; u < TU; ++u) {
        const int e = (int)threadIdx.x + 256 * u;
        v[u] = src[(int64_t)(e / TB) * ld + e % TB];
    }
}

__device__ __forceinline__ void tile_put(double (*S)[TB + 1], const double (&v)[TU]) {
#pragma unroll
    for (int u = 0; u < TU; ++u) {
        const int e = (int)threadIdx.x + 256 * u;
        S[e / TB][e % TB] = v[u];
    }
}

__device__ __forceinline__ void tile_load(double (*S)[TB + 1], const double *src, int ld) {
    double v[TU];
    tile_fetch(src, ld, v);
    tile_put(S, v);
}

// transposed: S[c][r] = src[r][c]
__device__ __forceinline__ void tile_load_t(double (*S)[TB + 1], const double *src, int ld) {
    double v[TU];
    tile_fetch(src, ld, v);
#pragma unroll
    for (int u = 0; u < TU; ++u) {
        const int e = (int)threadIdx.x + 256 * u;
        S[e % TB][e / TB] = v[u];
    }
}

__device__ __forceinline__ void tile_store(double *dst, int ld, const double (*S)[TB + 1]) {
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x)
        dst[(int64_t)(e / TB) * ld + e % TB] = S[e / TB][e % TB];
}

// One tile column of the right-looking blocked Cholesky, all matrices of the
// batch at once (grid x).  Launch p >= 0 covers the tiles (I, J) with
// p < J <= I < PR (grid y, lower triangle by rows):
//   L_Ip = G_Ip W_p^T and L_Jp = G_Jp W_p^T (each workgroup forms the two it
//   needs; the (I, p + 1) workgroups store L_Ip in Lf),
//   G_IJ -= L_Ip L_Jp^T,
// and the workgroup of the new diagonal tile (p + 1, p + 1) factors it at once
// into Lf and its inverse into W.  Launch p = -1 factors tile (0, 0).  In the
// greedy form (PR = P + 1) tile row P is the right-hand side, whose last slot
// (P, P) only completes L_{P, P-1}; G keeps the updated, unscaled tiles.
__global__ __launch_bounds__(256) void k_big_chol_col(double *__restrict__ G,
                                                      double *__restrict__ Lf, int ld,
                                                      int64_t mstride, int p, int P,
                                                      double *__restrict__ W,
                                                      int32_t *__restrict__ fail,
                                                      Ctrl *__restrict__ ctrl) {
    if (ctrl_done(ctrl)) return;
    __shared__ double sW[TB][TB + 1], sA[TB][TB + 1], sB[TB][TB + 1], sT[TB][TB + 1];
    const int bt = blockIdx.x;
    int I = 0, J = 0;
    if (p >= 0) {
        const int f = blockIdx.y;
        int a = 0;
        while ((a + 1) * (a + 2) / 2 <= f) ++a;
        I = p + 1 + a;
        J = p + 1 + (f - a * (a + 1) / 2);
        if (J >= P && J != p + 1) return;   // unused right-hand-side slot
    }
    const bool rhs_slot = J >= P;
    double *Gb = G + (int64_t)bt * mstride;
    double *Lb = Lf + (int64_t)bt * mstride;
    // every tile this workgroup reads is fetched before any is stored to LDS
    // (one memory latency instead of one per tile)
    {
        double vw[TU], va[TU], vb[TU], vt[TU];
        if (p >= 0) {
            tile_fetch(W + ((int64_t)bt * P + p) * TB * TB, TB, vw);
            tile_fetch(Gb + (int64_t)(I * TB) * ld + p * TB, ld, va);
            if (J != I) tile_fetch(Gb + (int64_t)(J * TB) * ld + p * TB, ld, vb);
        }
        if (!rhs_slot) tile_fetch(Gb + (int64_t)(I * TB) * ld + J * TB, ld, vt);
        if (p >= 0) {
            tile_put(sW, vw);
            tile_put(sA, va);
            if (J != I) tile_put(sB, vb);
        }
        if (!rhs_slot) tile_put(sT, vt);
    }
    __syncthreads();
    if (p >= 0) {
        const dvec4 li = mm32_abt(sA, sW);
        dvec4 lj = li;
        if (J != I) lj = mm32_abt(sB, sW);
        __syncthreads();
        st32(sA, li);
        if (J != I) st32(sB, lj);
        __syncthreads();
        if (J == p + 1) tile_store(Lb + (int64_t)(I * TB) * ld + p * TB, ld, sA);
        if (rhs_slot) return;
        const dvec4 u = mm32_abt(sA, (J != I) ? sB : sA);
        {
            const int w = threadIdx.x >> 6, R = w >> 1, C = w & 1;
            const int l = threadIdx.x & 63, lci = l & 15, lk = l >> 4;
#pragma unroll
            for (int r = 0; r < 4; ++r) sT[R * 16 + lk + 4 * r][C * 16 + lci] -= u[r];
        }
        __syncthreads();
    }
    if (I == J && (p < 0 || J == p + 1)) {
        // the new diagonal tile: factor in place, inverse into sW
        const bool ok = tile_factor32(sT, sW);
        if (threadIdx.x == 0 && !ok) {
            if (fail) *fail = 1;
            if (ctrl) {
                ctrl->status = RORBK_ERR_NOT_SPD;
                ctrl->done = 1;
            }
        }
        tile_store(Lb + (int64_t)(J * TB) * ld + J * TB, ld, sT);
        double *Wj = W + ((int64_t)bt * P + J) * TB * TB;
        for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) Wj[e] = sW[e / TB][e % TB];
    } else {
        tile_store(Gb + (int64_t)(I * TB) * ld + J * TB, ld, sT);
    }
}

// X = A B^T for 32 x 32 tiles staged in LDS: thread t (of 256) computes row
// t / 8, columns 4 (t % 8) .. +3, each a 32-term sum in k order.
__device__ __forceinline__ void tile_abt(const double (*A)[TB + 1], const double (*B)[TB + 1],
                                         double out[4]) {
    const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        double s = 0.0;
#pragma unroll
        for (int k = 0; k < TB; ++k) s = __builtin_fma(A[r][k], B[c0 + u][k], s);
        out[u] = s;
    }
}

// Row of tiles I of X = L^{-1} (L from Lf): X_II = W_I and, for J < I,
// X_IJ = -W_I sum_{k=J}^{I-1} L_Ik X_kJ (sum in k order).
__global__ __launch_bounds__(256) void k_big_invrow(const double *__restrict__ Lf, int ld, int I,
                                                    const double *__restrict__ W, int P,
                                                    double *__restrict__ X) {
    __shared__ double sA[TB][TB + 1], sB[TB][TB + 1];
    const int bt = blockIdx.x, J = blockIdx.y;
    const int64_t ms = (int64_t)ld * ld;
    const double *Lb = Lf + (int64_t)bt * ms;
    double *Xb = X + (int64_t)bt * ms;
    const double *WI = W + ((int64_t)bt * P + I) * TB * TB;
    const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
    double *dst = Xb + (int64_t)(I * TB) * ld + J * TB;
    if (J == I) {
#pragma unroll
        for (int u = 0; u < 4; ++u) dst[(int64_t)r * ld + c0 + u] = WI[r * TB + c0 + u];
        return;
    }
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = J; k < I; ++k) {
        tile_load(sA, Lb + (int64_t)(I * TB) * ld + k * TB, ld);     // L_Ik
        tile_load_t(sB, Xb + (int64_t)(k * TB) * ld + J * TB, ld);   // X_kJ^T
        __syncthreads();
        double out[4];
        tile_abt(sA, sB, out);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += out[u];
        __syncthreads();
    }
    // -W_I acc as A B^T with A = W_I, B = acc^T
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) sA[e / TB][e % TB] = WI[e];
#pragma unroll
    for (int u = 0; u < 4; ++u) sB[c0 + u][r] = acc[u];
    __syncthreads();
    double out[4];
    tile_abt(sA, sB, out);
#pragma unroll
    for (int u = 0; u < 4; ++u) dst[(int64_t)r * ld + c0 + u] = -out[u];
}

// Stored inverse of block t0 + bt: H = X^T X with H_IJ = sum_{k >= I} X_kI^T
// X_kJ (J <= I, k order), written in full as the block's rows x rows row-major
// array at its offset in H (fixedK > 0, column form: fixedK x fixedK at
// t * fixedK^2); the mirrored entries come from the lower ones.
__global__ __launch_bounds__(256) void k_big_xtx(const double *__restrict__ X, int ld, int P,
                                                 int64_t t0, int64_t q, int64_t rem, int fixedK,
                                                 double *__restrict__ H) {
    __shared__ double sA[TB][TB + 1], sB[TB][TB + 1];
    const int bt = blockIdx.x, f = blockIdx.y;
    int I = 0;
    while ((I + 1) * (I + 2) / 2 <= f) ++I;
    const int J = f - I * (I + 1) / 2;
    const double *Xb = X + (int64_t)bt * ld * ld;
    double acc[4] = {0.0, 0.0, 0.0, 0.0};
    for (int k = I; k < P; ++k) {
        tile_load_t(sA, Xb + (int64_t)(k * TB) * ld + I * TB, ld);   // X_kI^T
        tile_load_t(sB, Xb + (int64_t)(k * TB) * ld + J * TB, ld);   // X_kJ^T
        __syncthreads();
        double out[4];
        tile_abt(sA, sB, out);
#pragma unroll
        for (int u = 0; u < 4; ++u) acc[u] += out[u];
        __syncthreads();
    }
    const int64_t t = t0 + bt;
    const int K = fixedK > 0 ? fixedK : blk_rows(t, q, rem);
    double *Hb = H + (fixedK > 0 ? t * (int64_t)fixedK * fixedK : blk_hoff(t, q, rem));
    const int r = threadIdx.x >> 3, c0 = (threadIdx.x & 7) * 4;
#pragma unroll
    for (int u = 0; u < 4; ++u) {
        const int gi = I * TB + r, gj = J * TB + c0 + u;
        if (gi < K && gj < K && gj <= gi) {
            Hb[(int64_t)gi * K + gj] = acc[u];
            Hb[(int64_t)gj * K + gi] = acc[u];
        }
    }
}

// Backward solve L^T y = z of the greedy system (one workgroup), z being the
// right-hand-side row of the factor, two tile columns (lo = hi - 1, hi) per
// step from the last: t = z_{lo,hi} - sum_{k > hi} L_k,{lo,hi}^T y_k (thread
// (c, s) sums the rows s, s + 16, ... of column c of the 64-wide block; the 16
// row segments are added in order), then y_hi = W_hi^T t_hi,
// t_lo -= L_{hi,lo}^T y_hi and y_lo = W_lo^T t_lo.  Every load of a step (its
// column block of L, W_hi, W_lo, L_{hi,lo}) is issued together.  With an odd
// number of tile columns the first step (from the bottom) takes one.
constexpr int BS_T = 1024;
constexpr int BS_R = 32;   // rows per thread per round

__global__ __launch_bounds__(BS_T) void k_big_bsolve(const double *__restrict__ Lf, int ld, int P,
                                                     const double *__restrict__ W, int K,
                                                     double *__restrict__ y,
                                                     const Ctrl *__restrict__ ctrl) {
    if (ctrl_done(ctrl)) return;
    __shared__ double z[BIGB];
    __shared__ double part[2 * TB][17];
    __shared__ double sWh[TB][TB + 1], sWl[TB][TB + 1], sLhl[TB][TB + 1];
    __shared__ double t[2 * TB];
    const int tid = threadIdx.x, c = tid & (2 * TB - 1), sg = tid >> 6;
    for (int i = tid; i < P * TB; i += BS_T) z[i] = Lf[(int64_t)ld * ld + i];
    __syncthreads();
    int hi = P - 1;
    while (hi >= 0) {
        const int lo = ((P - 1 - hi) == 0 && (P & 1)) ? -1 : hi - 1;   // odd P: single first step
        const int c0 = (lo >= 0 ? lo : hi) * TB;                       // first column of the step
        const int ncol = (lo >= 0) ? 2 * TB : TB;
        const double wh = W[(int64_t)hi * TB * TB + tid];
        const double wl = (lo >= 0) ? W[(int64_t)lo * TB * TB + tid] : 0.0;
        const double lhl = (lo >= 0) ? Lf[(int64_t)(hi * TB + (tid >> 5)) * ld + lo * TB + (tid & 31)] : 0.0;
        double s = 0.0;
        const int nr = (P - hi - 1) * TB;          // rows below the step's diagonal tiles
        if (c < ncol) {
            for (int u0 = 0; u0 < nr; u0 += 16 * BS_R) {
                double gv[BS_R];
#pragma unroll
                for (int u = 0; u < BS_R; ++u) {
                    const int rr = u0 + sg + 16 * u;
                    gv[u] = (rr < nr) ? Lf[(int64_t)((hi + 1) * TB + rr) * ld + c0 + c] : 0.0;
                }
#pragma unroll
                for (int u = 0; u < BS_R; ++u) {
                    const int rr = u0 + sg + 16 * u;
                    if (rr < nr) s = __builtin_fma(gv[u], z[(hi + 1) * TB + rr], s);
                }
            }
        }
        part[c][sg] = s;
        sWh[tid >> 5][tid & 31] = wh;
        sWl[tid >> 5][tid & 31] = wl;
        sLhl[tid >> 5][tid & 31] = lhl;
        __syncthreads();
        // the 16 segment sums of each column by a fixed butterfly (16 lanes per column)
        {
            const int cc = tid >> 4, q2 = tid & 15;
            double v = group_sum(part[cc][q2], 16);
            if (q2 == 0 && cc < ncol) t[cc] = z[c0 + cc] - v;
        }
        __syncthreads();
        // 32 x 32 products below: output j by the 32 lanes (j, q), q summed by a
        // fixed butterfly
        const int oj = tid >> 5, oq = tid & 31;
        const int oh = ncol - TB;
        {   // y_hi = W_hi^T t_hi
            const double v = group_sum(sWh[oq][oj] * t[oh + oq], 32);
            if (oq == 0) z[hi * TB + oj] = v;
        }
        __syncthreads();
        if (lo >= 0) {
            {   // t_lo -= L_{hi,lo}^T y_hi
                const double v = group_sum(sLhl[oq][oj] * z[hi * TB + oq], 32);
                __syncthreads();
                if (oq == 0) t[oj] -= v;
            }
            __syncthreads();
            {   // y_lo = W_lo^T t_lo
                const double v = group_sum(sWl[oq][oj] * t[oq], 32);
                if (oq == 0) z[lo * TB + oj] = v;
            }
            __syncthreads();
        }
        hi = (lo >= 0) ? lo - 1 : hi - 1;
    }
    for (int i = tid; i < K; i += BS_T) y[i] = z[i];
}

// --------------------------------------------------------------- steps ----
// Row set size and start of a RowSel.
__device__ __forceinline__ void sel_rows(const RowSel &s, const int32_t *tau, int64_t q,
                                         int64_t rem, int *cnt, int64_t *start) {
    *cnt = 0;
    *start = 0;
    if (s.kind == 0) {
        const int t = tau[s.tau_index];
        *start = blk_start(t, q, rem);
        *cnt = blk_rows(t, q, rem);
    } else if (s.kind == 1) {
        *cnt = s.count;
    }
}

__device__ __forceinline__ int64_t sel_row(const RowSel &s, int64_t start, int i) {
    return (s.kind == 1) ? (int64_t)s.idx[i] : start + i;
}

// r_S = b_S - sum_ch Pin[ch][.] for the fixed block tau[tau_index], 16 rows
// per workgroup, 16 lanes per row over the chunks, fixed butterfly; with
// b == NULL (adjoint) r_S = -sum.
template <typename V>
__global__ __launch_bounds__(256) void k_big_r(const int32_t *__restrict__ tau, int64_t tau_index,
                                               int64_t q, int64_t rem, const V *__restrict__ b,
                                               const double *__restrict__ Pin, int nch, int bmax,
                                               double *__restrict__ r,
                                               const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    const int t = tau[tau_index];
    const int cnt = blk_rows(t, q, rem);
    const int64_t cst = blk_start(t, q, rem);
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
    double s = 0.0;
    if (i < cnt) {
        constexpr int U = 8;
        for (int cb = l; cb < nch; cb += U * 16) {
            double v[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int c = cb + 16 * u;
                v[u] = (c < nch) ? Pin[(int64_t)c * bmax + i] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) s += v[u];
        }
    }
    s = group_sum(s, 16);
    if (i < cnt && l == 0) r[i] = (b ? (double)b[cst + i] : 0.0) - s;
}

// y = H_t r for the fixed block tau[tau_index] (H_t symmetric, read by rows),
// 4 rows per workgroup, one wave per row, fixed butterfly.  With gb set
// (adjoint), gb[S] -= y.
template <typename V>
__global__ __launch_bounds__(256) void k_big_y(const double *__restrict__ H,
                                               const int32_t *__restrict__ tau, int64_t tau_index,
                                               int64_t q, int64_t rem,
                                               const double *__restrict__ r,
                                               double *__restrict__ y, V *__restrict__ gb,
                                               const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double sr[BIGB];
    const int t = tau[tau_index];
    const int cnt = blk_rows(t, q, rem);
    const int64_t cst = blk_start(t, q, rem);
    for (int j = threadIdx.x; j < cnt; j += blockDim.x) sr[j] = r[j];
    __syncthreads();
    const double *Hb = H + blk_hoff(t, q, rem);
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    double s = 0.0;
    if (i < cnt) {
        const double *row = Hb + (int64_t)i * cnt;
        constexpr int U = 8;
        for (int jb = l; jb < cnt; jb += U * 64) {
            double hv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + 64 * u;
                hv[u] = (j < cnt) ? row[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + 64 * u;
                if (j < cnt) s = __builtin_fma(hv[u], sr[j], s);
            }
        }
    }
    s = group_sum(s, 64);
    if (i < cnt && l == 0) {
        y[i] = s;
        if (gb) gb[cst + i] -= (V)s;
    }
}

struct BigP {
    const void *A;
    int64_t ld, n, q, rem;
    const int32_t *tau;
    RowSel cur;
    int upd;              // 0: no update (first partial products)
    const double *y;      // y of the current step (cur's row order)
    void *x;              // iterate (vector type)
    void *xold;           // copy of x taken by the update kernel
    void *dxp;            // column partial sums [row chunk][n]
    void *gb;             // adjoint, gathered sets: gb[S] -= y
    RowSel nxt;
    double *Pout;         // [column chunk][bmax]
    int bmax;
    const double *dx;     // column form: the step's correction (x_new = xold + dx)
    const Ctrl *ctrl;
};

// Update partials: workgroup (w, rc) takes the 128 columns of chunk w and the
// rows rc*RCH .. +RCH of the current set: dxp[rc][cols] = sum over those rows
// (thread g sums rows g, g+G, ..., then the G groups in order) of A[row, cols]
// y_row.  Chunk row 0 also copies x[cols] to xold for the apply kernel.
template <typename T, typename V, bool AL>
__global__ __launch_bounds__(BIG_T) void k_big_upd(BigP p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int NV = 128 / VW;
    constexpr int G = BIG_T / NV;
    constexpr int RCH = big_rch<T>();
    if (p.ctrl->done) return;
    int cnt;
    int64_t cst;
    sel_rows(p.cur, p.tau, p.q, p.rem, &cnt, &cst);
    const int r0 = blockIdx.y * RCH;
    if (r0 >= cnt) return;
    const T *__restrict__ A = (const T *)p.A;
    const V *__restrict__ x = (const V *)p.x;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;
    const int64_t c0 = (int64_t)blockIdx.x * 128;
    const int64_t c1 = (c0 + 128 < p.n) ? c0 + 128 : p.n;
    const int64_t col = c0 + (int64_t)v * VW;
    uvec4 ua[BIG_RPT];
    double yv[BIG_RPT];
    const uvec4 zero4 = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < BIG_RPT; ++u) {
        const int i = r0 + g + G * u;
        const bool live = i < cnt;
        const int64_t row = live ? sel_row(p.cur, cst, i) : 0;
        ua[u] = load_raw_sel<T, AL>(A + row * p.ld, col, c1, live, A, c0);
        yv[u] = live ? p.y[i] : 0.0;
    }
    if (blockIdx.y == 0)
        for (int64_t c = c0 + tid; c < c1; c += BIG_T) ((V *)p.xold)[c] = x[c];
    if (p.gb && p.cur.kind == 1 && blockIdx.x == 0 && blockIdx.y == 0)
        for (int i = tid; i < cnt; i += BIG_T) ((V *)p.gb)[p.cur.idx[i]] -= (V)p.y[i];
    V acc[VW];
#pragma unroll
    for (int e = 0; e < VW; ++e) acc[e] = (V)0;
#pragma unroll
    for (int u = 0; u < BIG_RPT; ++u) {
        V a[VW];
        cvt_raw<T, V>(ua[u], a);
        const V yi = (V)yv[u];
#pragma unroll
        for (int e = 0; e < VW; ++e) acc[e] = fmaT(a[e], yi, acc[e]);
    }
    __shared__ V s_red[G][128];
#pragma unroll
    for (int e = 0; e < VW; ++e) s_red[g][v * VW + e] = acc[e];
    __syncthreads();
    if (tid < 128 && c0 + tid < c1) {
        V s = (V)0;
        for (int gg = 0; gg < G; ++gg) s += s_red[gg][tid];
        ((V *)p.dxp)[(int64_t)blockIdx.y * p.n + c0 + tid] = s;
    }
}

// Apply and next products: workgroup (w, rc) forms x_new[cols] = xold[cols] +
// sum_rc' dxp[rc'][cols] (rc' order), or xold + dx for the column form (x
// itself if there is no update), chunk
// row 0 writes it to x, and every workgroup produces the partial products
// Pout[w][i] = A[row_i, cols] . x_new[cols] of the next rows i in its chunk
// (lane sums by a fixed butterfly).
template <typename T, typename V, bool AL>
__global__ __launch_bounds__(BIG_T) void k_big_apply(BigP p) {
    constexpr int VW = Tr<T>::VW;
    constexpr int NV = 128 / VW;
    constexpr int G = BIG_T / NV;
    constexpr int RCH = big_rch<T>();
    if (p.ctrl->done) return;
    int cnt, ncnt;
    int64_t cst, nst;
    sel_rows(p.cur, p.tau, p.q, p.rem, &cnt, &cst);
    sel_rows(p.nxt, p.tau, p.q, p.rem, &ncnt, &nst);
    const T *__restrict__ A = (const T *)p.A;
    V *__restrict__ x = (V *)p.x;
    const int tid = threadIdx.x, g = tid / NV, v = tid % NV;
    const int64_t c0 = (int64_t)blockIdx.x * 128;
    const int64_t c1 = (c0 + 128 < p.n) ? c0 + 128 : p.n;
    const int64_t col = c0 + (int64_t)v * VW;
    const int r0 = blockIdx.y * RCH;
    // next rows' loads first: they do not depend on x
    uvec4 un[BIG_RPT];
    const uvec4 zero4 = {0u, 0u, 0u, 0u};
#pragma unroll
    for (int u = 0; u < BIG_RPT; ++u) {
        const int i = r0 + g + G * u;
        const bool live = i < ncnt;
        const int64_t row = live ? sel_row(p.nxt, nst, i) : 0;
        un[u] = load_raw_sel<T, AL>(A + row * p.ld, col, c1, live, A, c0);
    }
    __shared__ V s_x[128];
    if (tid < 128) {
        const int64_t c = c0 + tid;
        V xv = (V)0;
        if (c < c1) {
            if (p.upd && p.dx) {
                xv = ((const V *)p.xold)[c] + (V)p.dx[c];
                if (blockIdx.y == 0) x[c] = xv;
            } else if (p.upd && cnt > 0) {
                const int nrc = (cnt + RCH - 1) / RCH;
                V s = (V)0;
                for (int rc = 0; rc < nrc; ++rc) s += ((const V *)p.dxp)[(int64_t)rc * p.n + c];
                xv = ((const V *)p.xold)[c] + s;
                if (blockIdx.y == 0) x[c] = xv;
            } else {
                xv = x[c];
            }
        }
        s_x[tid] = xv;
    }
    __syncthreads();
    if (r0 >= ncnt) return;
#pragma unroll
    for (int u = 0; u < BIG_RPT; ++u) {
        const int i = r0 + g + G * u;
        V a[VW];
        cvt_raw<T, V>(un[u], a);
        V acc = (V)0;
#pragma unroll
        for (int e = 0; e < VW; ++e)
            if (col + e < c1) acc = fmaT(a[e], s_x[v * VW + e], acc);
        acc = group_sum(acc, NV);
        if (i < ncnt && v == 0) p.Pout[(int64_t)blockIdx.x * p.bmax + i] = (double)acc;
    }
}

// ------------------------------------------------------------ greedy Gram --
// Lower 32 x 32 tiles of A_I A_I^T (the greedy block's Gram) on FP64 MFMA for
// large greedy sets: grid x = tiles, grid y = column chunks; each wave holds
// the 16 x 16 sub-tiles of its tile over a quarter of the chunk's columns, so
// every row value it loads feeds two MFMA products (half the cache traffic of
// 16 x 16 tiles).  The four waves are summed in wave order.  Output: packed
// lower partials Gpart[chunk][pk(i, j)].
template <typename T, bool AL>
__global__ __launch_bounds__(256) void k_gram32(const T *__restrict__ A, int64_t ld, int64_t n,
                                                const int32_t *__restrict__ idx, int K, int64_t wg,
                                                double *__restrict__ Gpart,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    constexpr int VW = Tr<T>::VW;
    constexpr int E = (sizeof(T) == 8) ? 4 : VW;   // columns per lane per macro step
    constexpr int NL = E / VW;                      // 16-byte loads per row per step
    constexpr int U = (sizeof(T) == 8) ? 2 : 4;     // macro steps in flight
    const int nt = (K + 31) / 32;
    int bi, bj;
    tile_of(blockIdx.x, nt, &bi, &bj);
    const int64_t c0 = (int64_t)blockIdx.y * wg;
    const int64_t c1 = (c0 + wg < n) ? c0 + wg : n;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    const int64_t stepc = 4 * E;
    const int64_t span = ((c1 - c0 + 4 * stepc - 1) / (4 * stepc)) * stepc;
    const int64_t wa = c0 + w * span;
    const int64_t wb = (wa + span < c1) ? wa + span : c1;
    const bool same = (bi == bj);
    const T *pa[2], *pb[2];
    bool va[2], vb[2];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2) {
        const int ia = bi * 32 + s2 * 16 + li, ib = bj * 32 + s2 * 16 + li;
        va[s2] = ia < K;
        vb[s2] = ib < K;
        pa[s2] = A + (va[s2] ? (int64_t)idx[ia] : 0) * ld;
        pb[s2] = A + (vb[s2] ? (int64_t)idx[ib] : 0) * ld;
    }
    const dvec4 z4 = {0.0, 0.0, 0.0, 0.0};
    dvec4 acc[2][2] = {{z4, z4}, {z4, z4}};
    const uvec4 zu = {0u, 0u, 0u, 0u};
    for (int64_t c = wa; c < wb; c += 4 * E * U) {
        uvec4 xa[U][2][NL], xb[U][2][NL];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int64_t col = c + (int64_t)u * 4 * E + (int64_t)g * E;
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                const int64_t cc = col + h * VW;
#pragma unroll
                for (int s2 = 0; s2 < 2; ++s2) {
                    xa[u][s2][h] = load_raw_sel<T, AL>(pa[s2], cc, wb, va[s2], pa[s2], wa);
                    xb[u][s2][h] = load_raw_sel<T, AL>(pb[s2], cc, wb, !same && vb[s2], pb[s2], wa);
                }
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u)
#pragma unroll
            for (int h = 0; h < NL; ++h) {
                double a0[VW], a1[VW], b0[VW], b1[VW];
                cvt_raw<T, double>(xa[u][0][h], a0);
                cvt_raw<T, double>(xa[u][1][h], a1);
                if (same) {
#pragma unroll
                    for (int e = 0; e < VW; ++e) { b0[e] = a0[e]; b1[e] = a1[e]; }
                } else {
                    cvt_raw<T, double>(xb[u][0][h], b0);
                    cvt_raw<T, double>(xb[u][1][h], b1);
                }
#pragma unroll
                for (int e = 0; e < VW; ++e) {
                    acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], b0[e], acc[0][0], 0, 0, 0);
                    acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], b0[e], acc[1][0], 0, 0, 0);
                    acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a1[e], b1[e], acc[1][1], 0, 0, 0);
                    if (!same)
                        acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(a0[e], b1[e], acc[0][1], 0, 0, 0);
                }
            }
    }
    __shared__ double red[4][16][64];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][(s2 * 2 + t2) * 4 + r][lane] = acc[s2][t2][r];
    __syncthreads();
    if (w == 0) {
        const int KP = K * (K + 1) / 2;
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q2 = (s2 * 2 + t2) * 4 + r;
                    const double v = ((red[0][q2][lane] + red[1][q2][lane]) + red[2][q2][lane]) +
                                     red[3][q2][lane];
                    const int ii = bi * 32 + s2 * 16 + (lane >> 4) + 4 * r;
                    const int jj = bj * 32 + t2 * 16 + li;
                    if (ii < K && jj <= ii) Gpart[(int64_t)blockIdx.y * KP + pk(ii, jj)] = v;
                }
    }
}

// The same Gram on 64 x 64 tiles for FP64 rows (gram_tiles.h): every row value
// a wave loads feeds four MFMA products instead of two, half the cache
// traffic per flop of k_gram32, with the same partials.  Grid x = lower 64 x
// 64 tiles, grid y = column chunks.
template <typename T, bool AL>
__global__ __launch_bounds__(256) void k_gram64(const T *__restrict__ A, int64_t ld, int64_t n,
                                                const int32_t *__restrict__ idx, int K, int64_t wg,
                                                double *__restrict__ Gpart,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    const int nt = (K + 63) / 64;
    int bi, bj;
    tile_of(blockIdx.x, nt, &bi, &bj);
    const int64_t c0 = (int64_t)blockIdx.y * wg;
    const int64_t c1 = (c0 + wg < n) ? c0 + wg : n;
    const int li = threadIdx.x & 15;
    const T *pa[4], *pb[4];
    bool va[4], vb[4];
#pragma unroll
    for (int s2 = 0; s2 < 4; ++s2) {
        const int ia = bi * 64 + s2 * 16 + li, ib = bj * 64 + s2 * 16 + li;
        va[s2] = ia < K;
        vb[s2] = ib < K;
        pa[s2] = A + (int64_t)idx[va[s2] ? ia : 0] * ld;
        pb[s2] = A + (int64_t)idx[vb[s2] ? ib : 0] * ld;
    }
    dvec4 acc[4][4];
    gram64_accumulate<T, AL>(pa, pb, va, vb, bi == bj, c0, c1, acc);
    gram64_store(acc, bi, bj, K, Gpart + (int64_t)blockIdx.y * ((int64_t)K * (K + 1) / 2));
}

template <typename T>
static hipError_t gram64_typed(const rorbk_handle_s *h, const void *A, int aligned,
                               const int32_t *idx, int K, double *Gpart, hipStream_t s) {
    const Layout &L = h->L;
    const int nt = (K + 63) / 64;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)L.nch_g);
    if (aligned)
        hipLaunchKernelGGL((k_gram64<T, true>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_gram64<T, false>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

template <typename T>
static hipError_t gram32_typed(const rorbk_handle_s *h, const void *A, int aligned,
                               const int32_t *idx, int K, double *Gpart, hipStream_t s) {
    const Layout &L = h->L;
    const int nt = (K + 31) / 32;
    dim3 grid((unsigned)(nt * (nt + 1) / 2), (unsigned)L.nch_g);
    if (aligned)
        hipLaunchKernelGGL((k_gram32<T, true>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    else
        hipLaunchKernelGGL((k_gram32<T, false>), grid, dim3(256), 0, s, (const T *)A, L.ld, L.n,
                           idx, K, L.wg, Gpart, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_gram_big(const rorbk_handle_s *h, const void *A, int dt, const int32_t *idx,
                           int K, double *Gpart, hipStream_t s) {
    const int al = h->aligned;
    if (dt == RORBK_F64 && gram64_for(h->L.dtype, K))
        return gram64_typed<double>(h, A, al, idx, K, Gpart, s);
    if (dt == RORBK_F64) return gram32_typed<double>(h, A, al, idx, K, Gpart, s);
    if (dt == RORBK_F32) return gram32_typed<float>(h, A, al, idx, K, Gpart, s);
    return gram32_typed<bf16_t>(h, A, al, idx, K, Gpart, s);
}

// ------------------------------------------------------------ column form --
// For blocks with at least as many rows as columns the update uses the
// column form of the regularised block solve (Sec. 3.1; Lemma 1 for the
// regularised system): A_S^T (A_S A_S^T + lambda I)^{-1} r equals
// (A_S^T A_S + lambda I)^{-1} A_S^T r, whose system is n x n instead of b x b.
// Stored inverses M_t = (A_t^T A_t + lambda I)^{-1} (n x n, block t at t n^2);
// a step forms g = A_S^T r_S (the update kernel with y = r_S), dx = M g, and
// x += dx in the apply kernel.

// Column Gram A_S^T A_S of a row set (lower 32 x 32 tiles of the n x n
// result on FP64 MFMA): the rows of block t0 + blockIdx.z (idx == NULL) or the
// gathered rows idx[0 .. cnt).  Grid x = tiles, y = row chunks of rch rows,
// z = batch.  Each wave sums a quarter of the chunk's rows, four rows (the
// MFMA's k) per step: lane (c, g) supplies row g of the step at column c of
// the tile.  The four waves are summed in order.  Output: packed lower
// partials G[(z * nchunk + chunk) * n(n+1)/2 + pk(i, j)].
template <typename T>
__global__ __launch_bounds__(256) void k_colgram(const T *__restrict__ A, int64_t ld, int n,
                                                 const int32_t *__restrict__ idx, int cnt_g,
                                                 int64_t t0, int64_t q, int64_t rem, int rch,
                                                 int nchunk, double *__restrict__ G,
                                                 const Ctrl *__restrict__ ctrl) {
    if (ctrl_done(ctrl)) return;
    constexpr int U = 4;   // row steps in flight
    const int nt = (n + 31) / 32;
    int bi, bj;
    tile_of(blockIdx.x, nt, &bi, &bj);
    int cnt;
    int64_t rs = 0;
    if (idx) {
        cnt = cnt_g;
    } else {
        const int64_t t = t0 + blockIdx.z;
        cnt = blk_rows(t, q, rem);
        rs = blk_start(t, q, rem);
    }
    const int r0 = blockIdx.y * rch;
    const int r1 = (r0 + rch < cnt) ? r0 + rch : cnt;
    const int w = threadIdx.x >> 6, lane = threadIdx.x & 63, li = lane & 15, g = lane >> 4;
    const int nrw = ((r1 - r0 + 15) / 16) * 4;   // rows per wave, a multiple of 4
    const int wr0 = r0 + w * nrw;
    const int wr1 = (wr0 + nrw < r1) ? wr0 + nrw : r1;
    const bool same = bi == bj;
    const int ca[2] = {bi * 32 + li, bi * 32 + 16 + li};
    const int cb[2] = {bj * 32 + li, bj * 32 + 16 + li};
    const dvec4 z4 = {0.0, 0.0, 0.0, 0.0};
    dvec4 acc[2][2] = {{z4, z4}, {z4, z4}};
    for (int r = wr0; r < wr1; r += 4 * U) {
        double xa[U][2], xb[U][2];
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const int rr = r + 4 * u + g;
            const bool valid = rr < wr1;
            const int64_t row = valid ? (idx ? (int64_t)idx[rr] : rs + rr) : 0;
            const T *pr = A + row * ld;
#pragma unroll
            for (int s2 = 0; s2 < 2; ++s2) {
                xa[u][s2] = (valid && ca[s2] < n) ? to_v<double>(pr[ca[s2]]) : 0.0;
                xb[u][s2] = (!same && valid && cb[s2] < n) ? to_v<double>(pr[cb[s2]]) : 0.0;
            }
        }
#pragma unroll
        for (int u = 0; u < U; ++u) {
            const double b0 = same ? xa[u][0] : xb[u][0];
            const double b1 = same ? xa[u][1] : xb[u][1];
            acc[0][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][0], b0, acc[0][0], 0, 0, 0);
            acc[1][0] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][1], b0, acc[1][0], 0, 0, 0);
            acc[1][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][1], b1, acc[1][1], 0, 0, 0);
            if (!same)
                acc[0][1] = __builtin_amdgcn_mfma_f64_16x16x4f64(xa[u][0], b1, acc[0][1], 0, 0, 0);
        }
    }
    __shared__ double red[4][16][64];
#pragma unroll
    for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
        for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
            for (int r = 0; r < 4; ++r) red[w][(s2 * 2 + t2) * 4 + r][lane] = acc[s2][t2][r];
    __syncthreads();
    if (w == 0) {
        const int64_t KP = (int64_t)n * (n + 1) / 2;
        double *out = G + ((int64_t)blockIdx.z * nchunk + blockIdx.y) * KP;
#pragma unroll
        for (int s2 = 0; s2 < 2; ++s2)
#pragma unroll
            for (int t2 = 0; t2 < 2; ++t2)
#pragma unroll
                for (int r = 0; r < 4; ++r) {
                    const int q2 = (s2 * 2 + t2) * 4 + r;
                    const double v = ((red[0][q2][lane] + red[1][q2][lane]) + red[2][q2][lane]) +
                                     red[3][q2][lane];
                    const int ii = bi * 32 + s2 * 16 + (lane >> 4) + 4 * r;
                    const int jj = bj * 32 + t2 * 16 + li;
                    if (ii < n && jj <= ii) out[pk(ii, jj)] = v;
                }
    }
}

// g_j = sum_rc dxp[rc][j] (rc order): A_I^T r_I from the update kernel's
// row-chunk partials, the right-hand side of the greedy column system.
template <typename V>
__global__ __launch_bounds__(256) void k_col_sum(const V *__restrict__ dxp, int nrc, int n,
                                                 double *__restrict__ g,
                                                 const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j >= n) return;
    double s = 0.0;
    for (int rc = 0; rc < nrc; ++rc) s += (double)dxp[(int64_t)rc * n + j];
    g[j] = s;
}

// Fixed block t = tau[tau_index], column form: g = sum_rc dxp[rc] (rc order,
// in LDS), dx = M_t g with one wave per row of M_t (symmetric, read by rows)
// and a fixed butterfly; 4 rows per workgroup.
template <typename V, int RCH>
__global__ __launch_bounds__(256) void k_col_dx(const double *__restrict__ H,
                                                const int32_t *__restrict__ tau, int64_t tau_index,
                                                int64_t q, int64_t rem, int n,
                                                const V *__restrict__ dxp, double *__restrict__ dx,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double sg[BIGB];
    const int t = tau[tau_index];
    const int nrc = (blk_rows(t, q, rem) + RCH - 1) / RCH;
    for (int j = threadIdx.x; j < n; j += blockDim.x) {
        double s = 0.0;
        for (int rc = 0; rc < nrc; ++rc) s += (double)dxp[(int64_t)rc * n + j];
        sg[j] = s;
    }
    __syncthreads();
    const double *M = H + (int64_t)t * n * n;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    double s = 0.0;
    if (i < n) {
        const double *row = M + (int64_t)i * n;
        constexpr int UU = 8;
        for (int jb = l; jb < n; jb += UU * 64) {
            double mv[UU];
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int j = jb + 64 * u;
                mv[u] = (j < n) ? row[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < UU; ++u) {
                const int j = jb + 64 * u;
                if (j < n) s = __builtin_fma(mv[u], sg[j], s);
            }
        }
    }
    s = group_sum(s, 64);
    if (i < n && l == 0) dx[i] = s;
}

// Column form, adjoint.  The adjoint of a step needs y = -(A_S A_S^T +
// lambda I)^{-1} A_S g' (g' the incoming cotangent of x), which the column
// form gives as y = -A_S v with v = (A_S^T A_S + lambda I)^{-1} g'.
// v = M_t g' for the fixed block tau[tau_index]: g' in LDS (as FP64), one wave
// per row of M_t, fixed butterfly.
template <typename V>
__global__ __launch_bounds__(256) void k_col_mv(const double *__restrict__ H,
                                                const int32_t *__restrict__ tau, int64_t tau_index,
                                                int n, const V *__restrict__ gx,
                                                double *__restrict__ v,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double sg[BIGB];
    for (int j = threadIdx.x; j < n; j += blockDim.x) sg[j] = (double)gx[j];
    __syncthreads();
    const int t = tau[tau_index];
    const double *M = H + (int64_t)t * n * n;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    double s = 0.0;
    if (i < n) {
        const double *row = M + (int64_t)i * n;
        for (int j = l; j < n; j += 64) s = __builtin_fma(row[j], sg[j], s);
    }
    s = group_sum(s, 64);
    if (i < n && l == 0) v[i] = s;
}

// y_i = -(A_S v)_i for the rows of a step (one wave per row, v in LDS, fixed
// butterfly), and gb[row_i] -= y_i.
template <typename T, typename V>
__global__ __launch_bounds__(256) void k_col_av(const T *__restrict__ A, int64_t ld, int n,
                                                RowSel rs, const int32_t *__restrict__ tau,
                                                int64_t q, int64_t rem,
                                                const double *__restrict__ v,
                                                double *__restrict__ y, V *__restrict__ gb,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    __shared__ double sv[BIGB];
    for (int j = threadIdx.x; j < n; j += blockDim.x) sv[j] = v[j];
    __syncthreads();
    int cnt;
    int64_t cst;
    sel_rows(rs, tau, q, rem, &cnt, &cst);
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6), l = threadIdx.x & 63;
    double s = 0.0;
    int64_t row = 0;
    if (i < cnt) {
        row = sel_row(rs, cst, i);
        const T *pr = A + row * ld;
        for (int j = l; j < n; j += 64) s = __builtin_fma(to_v<double>(pr[j]), sv[j], s);
    }
    s = group_sum(s, 64);
    if (i < cnt && l == 0) {
        y[i] = -s;
        gb[row] += (V)s;
    }
}

// g'_j as FP64, the right-hand side of the greedy column system in the adjoint.
template <typename V>
__global__ __launch_bounds__(256) void k_to_f64(const V *__restrict__ src, int n,
                                                double *__restrict__ dst,
                                                const Ctrl *__restrict__ ctrl) {
    if (ctrl->done) return;
    const int j = blockIdx.x * blockDim.x + threadIdx.x;
    if (j < n) dst[j] = (double)src[j];
}

// ------------------------------------------------------------ launchers --
// Factor `batch` padded matrices (rows x ld each, rows = ld or ld + TB) in
// G: L into Lf, every diagonal tile's inverse into W[bt * P + p].
hipError_t big_potrf(double *G, double *Lf, int ld, int rows, int batch, double *W,
                            int32_t *fail, Ctrl *ctrl, hipStream_t s) {
    const int P = ld / TB, PR = rows / TB;
    const int64_t ms = (int64_t)rows * ld;
    const int last = (PR > P) ? P - 1 : P - 2;
    for (int p = -1; p <= last; ++p) {
        const int nt = (p < 0) ? 1 : (PR - p - 1) * (PR - p) / 2;
        hipLaunchKernelGGL(k_big_chol_col, dim3(batch, nt), dim3(256), 0, s, G, Lf, ld, ms, p, P,
                           W, fail, ctrl);
    }
    return hipGetLastError();
}

// Stored inverses of every fixed block from packed Grams Gs[t][kp], in
// batches of blocks that keep the two padded work arrays near 1 GiB each
// (the second holds L, then L^{-1} is formed in the first).
hipError_t launch_big_block_inverses(const rorbk_handle_s *h, const double *Gs, int64_t kp,
                                     int32_t *d_fail, hipStream_t s) {
    const Layout &L = h->L;
    const int P = (int)((L.bmax + TB - 1) / TB), ld = P * TB;
    const int64_t ms = (int64_t)ld * ld;
    int64_t bmaxb = ((int64_t)1 << 27) / ms;   // 2^27 doubles = 1 GiB per array
    if (bmaxb < 1) bmaxb = 1;
    if (bmaxb > L.k) bmaxb = L.k;
    double *G = nullptr, *Lf = nullptr, *W = nullptr;
    hipError_t e = hipMallocAsync((void **)&G, sizeof(double) * (size_t)(bmaxb * ms), s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&Lf, sizeof(double) * (size_t)(bmaxb * ms), s);
    if (e == hipSuccess)
        e = hipMallocAsync((void **)&W, sizeof(double) * (size_t)(bmaxb * P * TB * TB), s);
    for (int64_t t0 = 0; t0 < L.k && e == hipSuccess; t0 += bmaxb) {
        const int batch = (int)((L.k - t0 < bmaxb) ? L.k - t0 : bmaxb);
        hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)((ms + 255) / 256), (unsigned)batch),
                           dim3(256), 0, s, Gs + t0 * kp, kp, (int64_t)0, 1, 0, t0, L.q, L.rem,
                           h->lambda, ld, ld, (const double *)nullptr, (const double *)nullptr, 0,
                           0, G, (const Ctrl *)nullptr);
        e = big_potrf(G, Lf, ld, ld, batch, W, d_fail, nullptr, s);
        if (e != hipSuccess) break;
        double *X = G;   // G is free once factored
        for (int I = 0; I < P; ++I)
            hipLaunchKernelGGL(k_big_invrow, dim3((unsigned)batch, I + 1), dim3(256), 0, s,
                               (const double *)Lf, ld, I, (const double *)W, P, X);
        hipLaunchKernelGGL(k_big_xtx, dim3((unsigned)batch, P * (P + 1) / 2), dim3(256), 0, s,
                           (const double *)X, ld, P, t0, L.q, L.rem, 0, h->d_H);
        e = hipGetLastError();
    }
    if (G) (void)hipFreeAsync(G, s);
    if (Lf) (void)hipFreeAsync(Lf, s);
    if (W) (void)hipFreeAsync(W, s);
    return e;
}

// The greedy block's system (A_I A_I^T + lambda I) y = rhs from the Gram
// partials: unpack with the right-hand-side row, factor (which also solves
// L z = rhs), backward solve.
hipError_t launch_big_chol_solve(const rorbk_handle_s *h, const double *Gpart, int K,
                                 const double *rI, const double *Pin, double *y, hipStream_t s) {
    const Layout &L = h->L;
    const int P = (K + TB - 1) / TB, ld = P * TB, rows = ld + TB;
    const int64_t KP = (int64_t)K * (K + 1) / 2, el = (int64_t)rows * ld;
    hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)((el + 255) / 256), 1), dim3(256), 0, s,
                       Gpart, (int64_t)0, KP, (int)L.nch_g, K, (int64_t)0, L.q, L.rem, h->lambda,
                       ld, rows, rI, Pin, (int)L.nch_u, (int)L.bmax, h->d_bigG,
                       (const Ctrl *)h->d_ctrl);
    hipError_t e = big_potrf(h->d_bigG, h->d_bigL, ld, rows, 1, h->d_bigW, nullptr, h->d_ctrl, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_big_bsolve, dim3(1), dim3(BS_T), 0, s, (const double *)h->d_bigL, ld, P,
                       (const double *)h->d_bigW, K, y, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

// Column form, setup: M_t = (A_t^T A_t + lambda I)^{-1} for every block, in
// batches: column Grams (row chunks of 256), padded unpack, factorisation,
// L^{-1} by tile rows, M = L^{-T} L^{-1} at t n^2.
template <typename T>
static hipError_t col_inverses_typed(const rorbk_handle_s *h, const void *A, int32_t *d_fail,
                                     hipStream_t s) {
    const Layout &L = h->L;
    const int n = (int)L.n;
    const int P = (n + TB - 1) / TB, ld = P * TB;
    const int64_t ms = (int64_t)ld * ld, KP = (int64_t)n * (n + 1) / 2;
    const int rch = 256;
    const int nchunk = (int)((L.bmax + rch - 1) / rch);
    const int64_t per = (ms > (int64_t)nchunk * KP) ? ms : (int64_t)nchunk * KP;
    int64_t bmaxb = ((int64_t)1 << 27) / per;
    if (bmaxb < 1) bmaxb = 1;
    if (bmaxb > L.k) bmaxb = L.k;
    double *G = nullptr, *Lf = nullptr, *W = nullptr, *Gs = nullptr;
    hipError_t e = hipMallocAsync((void **)&G, sizeof(double) * (size_t)(bmaxb * ms), s);
    if (e == hipSuccess) e = hipMallocAsync((void **)&Lf, sizeof(double) * (size_t)(bmaxb * ms), s);
    if (e == hipSuccess)
        e = hipMallocAsync((void **)&W, sizeof(double) * (size_t)(bmaxb * P * TB * TB), s);
    if (e == hipSuccess)
        e = hipMallocAsync((void **)&Gs, sizeof(double) * (size_t)(bmaxb * nchunk * KP), s);
    const unsigned tiles = (unsigned)(P * (P + 1) / 2);
    for (int64_t t0 = 0; t0 < L.k && e == hipSuccess; t0 += bmaxb) {
        const int batch = (int)((L.k - t0 < bmaxb) ? L.k - t0 : bmaxb);
        hipLaunchKernelGGL(k_colgram<T>, dim3(tiles, (unsigned)nchunk, (unsigned)batch), dim3(256),
                           0, s, (const T *)A, L.ld, n, (const int32_t *)nullptr, 0, t0, L.q,
                           L.rem, rch, nchunk, Gs, (const Ctrl *)nullptr);
        hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)((ms + 255) / 256), (unsigned)batch),
                           dim3(256), 0, s, (const double *)Gs, (int64_t)nchunk * KP, KP, nchunk,
                           n, t0, L.q, L.rem, h->lambda, ld, ld, (const double *)nullptr,
                           (const double *)nullptr, 0, 0, G, (const Ctrl *)nullptr);
        e = big_potrf(G, Lf, ld, ld, batch, W, d_fail, nullptr, s);
        if (e != hipSuccess) break;
        double *X = G;
        for (int I = 0; I < P; ++I)
            hipLaunchKernelGGL(k_big_invrow, dim3((unsigned)batch, I + 1), dim3(256), 0, s,
                               (const double *)Lf, ld, I, (const double *)W, P, X);
        hipLaunchKernelGGL(k_big_xtx, dim3((unsigned)batch, P * (P + 1) / 2), dim3(256), 0, s,
                           (const double *)X, ld, P, t0, L.q, L.rem, n, h->d_H);
        e = hipGetLastError();
    }
    if (G) (void)hipFreeAsync(G, s);
    if (Lf) (void)hipFreeAsync(Lf, s);
    if (W) (void)hipFreeAsync(W, s);
    if (Gs) (void)hipFreeAsync(Gs, s);
    return e;
}

hipError_t launch_col_block_inverses(const rorbk_handle_s *h, const void *A, int dt,
                                     int32_t *d_fail, hipStream_t s) {
    if (dt == RORBK_F64) return col_inverses_typed<double>(h, A, d_fail, s);
    if (dt == RORBK_F32) return col_inverses_typed<float>(h, A, d_fail, s);
    return col_inverses_typed<bf16_t>(h, A, d_fail, s);
}

// Column form, greedy step: g = A_I^T r_I (update kernel over the gathered
// rows with y = r_I, which also copies x for the apply kernel), the column
// Gram of the gathered rows, then (A_I^T A_I + lambda I) dx = g by the padded
// factorisation with g as its right-hand-side row and the backward solve.
template <typename T, typename V>
static hipError_t col_greedy_typed(const rorbk_handle_s *h, const void *A, int aligned, void *x,
                                   const int32_t *I, int K, const double *rI, double *dx,
                                   hipStream_t s) {
    const Layout &L = h->L;
    constexpr int RCH = big_rch<T>();
    const int n = (int)L.n;
    const int P = (n + TB - 1) / TB, ld = P * TB, rows = ld + TB;
    const int64_t KP = (int64_t)n * (n + 1) / 2, el = (int64_t)rows * ld;
    BigP p = {};
    p.A = A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.tau = h->d_tau;
    p.cur.kind = 1;
    p.cur.count = K;
    p.cur.idx = I;
    p.upd = 1;
    p.y = rI;
    p.x = x;
    p.xold = h->d_xold;
    p.dxp = h->d_dxp;
    p.nxt.kind = -1;
    p.bmax = (int)L.bmax;
    p.ctrl = h->d_ctrl;
    const unsigned nrc = (unsigned)((K + RCH - 1) / RCH);
    if (aligned)
        hipLaunchKernelGGL((k_big_upd<T, V, true>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
    else
        hipLaunchKernelGGL((k_big_upd<T, V, false>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
    hipLaunchKernelGGL(k_colgram<T>, dim3((unsigned)(P * (P + 1) / 2), (unsigned)L.nch_g, 1),
                       dim3(256), 0, s, (const T *)A, L.ld, n, I, K, (int64_t)0, L.q, L.rem,
                       (int)L.wg, (int)L.nch_g, h->d_G, (const Ctrl *)h->d_ctrl);
    hipLaunchKernelGGL(k_col_sum<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                       (const V *)h->d_dxp, (int)nrc, n, h->d_bigr, (const Ctrl *)h->d_ctrl);
    hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)((el + 255) / 256), 1), dim3(256), 0, s,
                       (const double *)h->d_G, (int64_t)0, KP, (int)L.nch_g, n, (int64_t)0, L.q,
                       L.rem, h->lambda, ld, rows, (const double *)h->d_bigr,
                       (const double *)nullptr, 0, 0, h->d_bigG, (const Ctrl *)h->d_ctrl);
    hipError_t e = big_potrf(h->d_bigG, h->d_bigL, ld, rows, 1, h->d_bigW, nullptr, h->d_ctrl, s);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_big_bsolve, dim3(1), dim3(BS_T), 0, s, (const double *)h->d_bigL, ld, P,
                       (const double *)h->d_bigW, n, dx, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_col_greedy(const rorbk_handle_s *h, const void *A, int dt, int aligned, int vec,
                             void *x, const int32_t *I, int K, const double *rI, double *dx,
                             hipStream_t s) {
    if (vec == VEC_F64) return col_greedy_typed<double, double>(h, A, aligned, x, I, K, rI, dx, s);
    if (dt == RORBK_F32) return col_greedy_typed<float, float>(h, A, aligned, x, I, K, rI, dx, s);
    return col_greedy_typed<bf16_t, float>(h, A, aligned, x, I, K, rI, dx, s);
}

// Column form, adjoint of one step: v = M g' (fixed block: stored M_t; greedy
// set: the factorised column system with g' as its right-hand side), then
// y = -A_S v and gb[S] -= y into yout.  The caller then applies x += A_S^T y.
template <typename T, typename V>
static hipError_t col_adj_typed(const rorbk_handle_s *h, const RowSel &rs, const void *gx,
                                void *gb, double *yout, hipStream_t s) {
    const Layout &L = h->L;
    const int n = (int)L.n;
    const int P = (n + TB - 1) / TB, ld = P * TB, rows = ld + TB;
    const int64_t KP = (int64_t)n * (n + 1) / 2, el = (int64_t)rows * ld;
    if (rs.kind == 0) {
        hipLaunchKernelGGL(k_col_mv<V>, dim3((unsigned)((n + 3) / 4)), dim3(256), 0, s,
                           (const double *)h->d_H, h->d_tau, rs.tau_index, n, (const V *)gx,
                           h->d_bigy, (const Ctrl *)h->d_ctrl);
    } else {
        hipLaunchKernelGGL(k_colgram<T>, dim3((unsigned)(P * (P + 1) / 2), (unsigned)L.nch_g, 1),
                           dim3(256), 0, s, (const T *)h->A, L.ld, n, rs.idx, rs.count,
                           (int64_t)0, L.q, L.rem, (int)L.wg, (int)L.nch_g, h->d_G,
                           (const Ctrl *)h->d_ctrl);
        hipLaunchKernelGGL(k_to_f64<V>, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s,
                           (const V *)gx, n, h->d_bigr, (const Ctrl *)h->d_ctrl);
        hipLaunchKernelGGL(k_big_unpack, dim3((unsigned)((el + 255) / 256), 1), dim3(256), 0, s,
                           (const double *)h->d_G, (int64_t)0, KP, (int)L.nch_g, n, (int64_t)0,
                           L.q, L.rem, h->lambda, ld, rows, (const double *)h->d_bigr,
                           (const double *)nullptr, 0, 0, h->d_bigG, (const Ctrl *)h->d_ctrl);
        hipError_t e = big_potrf(h->d_bigG, h->d_bigL, ld, rows, 1, h->d_bigW, nullptr,
                                 h->d_ctrl, s);
        if (e != hipSuccess) return e;
        hipLaunchKernelGGL(k_big_bsolve, dim3(1), dim3(BS_T), 0, s, (const double *)h->d_bigL, ld,
                           P, (const double *)h->d_bigW, n, h->d_bigy, (const Ctrl *)h->d_ctrl);
    }
    hipLaunchKernelGGL((k_col_av<T, V>), dim3((unsigned)((L.bmax + 3) / 4)), dim3(256), 0, s,
                       (const T *)h->A, L.ld, n, rs, (const int32_t *)h->d_tau, L.q, L.rem,
                       (const double *)h->d_bigy, yout, (V *)gb, (const Ctrl *)h->d_ctrl);
    return hipGetLastError();
}

hipError_t launch_col_adjoint(const rorbk_handle_s *h, const RowSel &rs, int vec, const void *gx,
                              void *gb, double *yout, hipStream_t s) {
    const int dt = h->L.dtype;
    if (vec == VEC_F64) return col_adj_typed<double, double>(h, rs, gx, gb, yout, s);
    if (dt == RORBK_F32) return col_adj_typed<float, float>(h, rs, gx, gb, yout, s);
    return col_adj_typed<bf16_t, float>(h, rs, gx, gb, yout, s);
}

template <typename T, typename V>
static hipError_t big_step_typed(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    constexpr int RCH = big_rch<T>();
    const double *y = nullptr;
    const double *dx = nullptr;
    if (h->col && a.ymode == 0) {
        // column form: r_S, g partials (update kernel with y = r_S), dx = M_t g
        const unsigned g16 = (unsigned)((L.bmax + 15) / 16);
        hipLaunchKernelGGL(k_big_r<V>, dim3(g16), dim3(256), 0, s, h->d_tau, a.cur.tau_index,
                           L.q, L.rem, (const V *)a.b, a.Pin, (int)L.nch_u, (int)L.bmax,
                           h->d_bigr, (const Ctrl *)h->d_ctrl);
        y = h->d_bigr;
        dx = h->d_bigy;
    } else if (h->col && a.ymode == 1) {
        dx = a.ygiven;   // the greedy column solve ran the update kernel already
    } else if (a.ymode == 3) {
        y = a.ygiven;    // y given, update x += A_S^T y through the column partials
    } else if (a.ymode == 0) {
        const unsigned g16 = (unsigned)((L.bmax + 15) / 16);
        hipLaunchKernelGGL(k_big_r<V>, dim3(g16), dim3(256), 0, s, h->d_tau, a.cur.tau_index,
                           L.q, L.rem, (const V *)a.b, a.Pin, (int)L.nch_u, (int)L.bmax,
                           h->d_bigr, (const Ctrl *)h->d_ctrl);
        hipLaunchKernelGGL(k_big_y<V>, dim3((unsigned)((L.bmax + 3) / 4)), dim3(256), 0, s,
                           (const double *)h->d_H,
                           h->d_tau, a.cur.tau_index, L.q, L.rem, (const double *)h->d_bigr,
                           h->d_bigy, (V *)a.gb, (const Ctrl *)h->d_ctrl);
        y = h->d_bigy;
    } else if (a.ymode == 1) {
        y = a.ygiven;
    }
    BigP p;
    p.A = a.A;
    p.ld = L.ld;
    p.n = L.n;
    p.q = L.q;
    p.rem = L.rem;
    p.tau = h->d_tau;
    p.cur = a.cur;
    p.upd = (a.ymode != 2) ? 1 : 0;   // ymode 3: gb was updated with y already
    p.y = y;
    p.x = a.x;
    p.xold = h->d_xold;
    p.dxp = h->d_dxp;
    p.gb = (a.ymode == 1) ? a.gb : nullptr;   // fixed blocks update gb in k_big_y
    p.nxt = a.nxt;
    p.Pout = a.Pout;
    p.bmax = (int)L.bmax;
    p.dx = nullptr;
    p.ctrl = h->d_ctrl;
    const unsigned nrc = (unsigned)((L.bmax + RCH - 1) / RCH);
    if (h->col && a.ymode == 0) {
        if (a.aligned)
            hipLaunchKernelGGL((k_big_upd<T, V, true>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
        else
            hipLaunchKernelGGL((k_big_upd<T, V, false>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
        hipLaunchKernelGGL((k_col_dx<V, RCH>), dim3((unsigned)((L.n + 3) / 4)), dim3(256), 0, s,
                           (const double *)h->d_H, h->d_tau, a.cur.tau_index, L.q, L.rem,
                           (int)L.n, (const V *)h->d_dxp, h->d_bigy, (const Ctrl *)h->d_ctrl);
    } else if (p.upd && (!h->col || a.ymode == 3)) {
        if (a.aligned)
            hipLaunchKernelGGL((k_big_upd<T, V, true>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
        else
            hipLaunchKernelGGL((k_big_upd<T, V, false>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
    }
    p.dx = dx;
    const unsigned nrc2 = (a.nxt.kind >= 0) ? nrc : 1u;
    if (a.aligned)
        hipLaunchKernelGGL((k_big_apply<T, V, true>), dim3(L.nch_u, nrc2), dim3(BIG_T), 0, s, p);
    else
        hipLaunchKernelGGL((k_big_apply<T, V, false>), dim3(L.nch_u, nrc2), dim3(BIG_T), 0, s, p);
    return hipGetLastError();
}

hipError_t launch_step_big(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    if (a.vec == VEC_F64) return big_step_typed<double, double>(h, a, s);
    if (a.dt == RORBK_F32) return big_step_typed<float, float>(h, a, s);
    return big_step_typed<bf16_t, float>(h, a, s);
}

}  // namespace rorbk
