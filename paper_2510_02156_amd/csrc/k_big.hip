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

// Cholesky factor and inverse of a 16 x 16 SPD block in LDS (row stride RS) on
// one wave, lane i & 15 holding row i: right-looking elimination with the
// columns broadcast by readlane; the block is overwritten by L (zeros above
// the diagonal) and Wl receives L^{-1}, column j by lane j (forward
// substitution, the earlier columns applied as they are found).
__device__ __forceinline__ void f16(double *S, int RS, double *Wl, bool &ok) {
    const int lane = threadIdx.x & 63, i = lane & 15;
    double a[16], rk[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) a[j] = (j <= i) ? S[i * RS + j] : 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) {
        const double d = bcast64(a[k], k);
        ok = ok && (d > 0.0) && isfinite(d);
        const double r = rsq_nr(d);
        rk[k] = r;
        a[k] = (i == k) ? d * r : a[k] * r;
#pragma unroll
        for (int j = k + 1; j < 16; ++j) a[j] = __builtin_fma(-a[k], bcast64(a[k], j), a[j]);
    }
    wsync();
    if (lane < 16) {
#pragma unroll
        for (int j = 0; j < 16; ++j) S[i * RS + j] = (j <= i) ? a[j] : 0.0;
    }
    wsync();
    double acc[16];
#pragma unroll
    for (int r = 0; r < 16; ++r) acc[r] = (r == i) ? 1.0 : 0.0;
#pragma unroll
    for (int c = 0; c < 16; ++c) {
        const double w = acc[c] * rk[c];
        acc[c] = w;
#pragma unroll
        for (int r = c + 1; r < 16; ++r) acc[r] = __builtin_fma(-S[r * RS + c], w, acc[r]);
    }
    if (lane < 16) {
#pragma unroll
        for (int r = 0; r < 16; ++r) Wl[r * RS + i] = acc[r];
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

__device__ __forceinline__ void tile_load(double (*S)[TB + 1], const double *src, int ld) {
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x)
        S[e / TB][e % TB] = src[(int64_t)(e / TB) * ld + e % TB];
}

// transposed: S[c][r] = src[r][c]
__device__ __forceinline__ void tile_load_t(double (*S)[TB + 1], const double *src, int ld) {
    for (int e = threadIdx.x; e < TB * TB; e += blockDim.x)
        S[e % TB][e / TB] = src[(int64_t)(e / TB) * ld + e % TB];
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
    if (p >= 0) {
        const double *Wp = W + ((int64_t)bt * P + p) * TB * TB;
        for (int e = threadIdx.x; e < TB * TB; e += blockDim.x) sW[e / TB][e % TB] = Wp[e];
        tile_load(sA, Gb + (int64_t)(I * TB) * ld + p * TB, ld);
        if (J != I) tile_load(sB, Gb + (int64_t)(J * TB) * ld + p * TB, ld);
    }
    if (!rhs_slot) tile_load(sT, Gb + (int64_t)(I * TB) * ld + J * TB, ld);
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
// array at its offset in H; the mirrored entries come from the lower ones.
__global__ __launch_bounds__(256) void k_big_xtx(const double *__restrict__ X, int ld, int P,
                                                 int64_t t0, int64_t q, int64_t rem,
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
    const int K = blk_rows(t, q, rem);
    double *Hb = H + blk_hoff(t, q, rem);
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
// right-hand-side row of the factor.  For each tile column p from the last:
// t = z_p - sum_{k > p} L_kp^T y_k (thread (r, s) sums the rows s, s + 32, ...
// of column r; the 32 row segments are added in order), then y_p = W_p^T t.
// Every load of a step (its column block of L, W_p) is issued together.
constexpr int BS_T = 1024;
constexpr int BS_R = 32;   // rows per thread per round

__global__ __launch_bounds__(BS_T) void k_big_bsolve(const double *__restrict__ Lf, int ld, int P,
                                                     const double *__restrict__ W, int K,
                                                     double *__restrict__ y,
                                                     const Ctrl *__restrict__ ctrl) {
    if (ctrl_done(ctrl)) return;
    __shared__ double z[BIGB];
    __shared__ double part[TB][TB + 1];
    __shared__ double sWp[TB][TB + 1];
    __shared__ double t[TB];
    const int tid = threadIdx.x, r = tid & (TB - 1), sg = tid >> 5;
    for (int i = tid; i < P * TB; i += BS_T) z[i] = Lf[(int64_t)ld * ld + i];
    __syncthreads();
    for (int p = P - 1; p >= 0; --p) {
        const double wv = W[(int64_t)p * TB * TB + tid];
        double s = 0.0;
        const int nr = P - p - 1;                 // tile rows below the diagonal
        for (int u0 = 0; u0 < nr; u0 += BS_R) {
            double gv[BS_R];
#pragma unroll
            for (int u = 0; u < BS_R; ++u) {
                const int c = (p + 1 + u0 + u) * TB + sg;
                gv[u] = (u0 + u < nr) ? Lf[(int64_t)c * ld + p * TB + r] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < BS_R; ++u) {
                const int c = (p + 1 + u0 + u) * TB + sg;
                if (u0 + u < nr) s = __builtin_fma(gv[u], z[c], s);
            }
        }
        part[r][sg] = s;
        sWp[tid >> 5][tid & 31] = wv;
        __syncthreads();
        if (tid < TB) {
            double v = z[p * TB + tid];
            for (int q2 = 0; q2 < TB; ++q2) v -= part[tid][q2];
            t[tid] = v;
        }
        __syncthreads();
        if (tid < TB) {
            double v = 0.0;
            for (int c = tid; c < TB; ++c) v = __builtin_fma(sWp[c][tid], t[c], v);
            z[p * TB + tid] = v;
        }
        __syncthreads();
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
// 16 rows per workgroup, 16 lanes per row, fixed butterfly.  With gb set
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
    const int i = blockIdx.x * 16 + (threadIdx.x >> 4), l = threadIdx.x & 15;
    double s = 0.0;
    if (i < cnt) {
        const double *row = Hb + (int64_t)i * cnt;
        constexpr int U = 16;
        for (int jb = l; jb < cnt; jb += U * 16) {
            double hv[U];
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + 16 * u;
                hv[u] = (j < cnt) ? row[j] : 0.0;
            }
#pragma unroll
            for (int u = 0; u < U; ++u) {
                const int j = jb + 16 * u;
                if (j < cnt) s = __builtin_fma(hv[u], sr[j], s);
            }
        }
    }
    s = group_sum(s, 16);
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
        ua[u] = (live && col < c1) ? load_raw<T, AL>(A + row * p.ld, col, c1) : zero4;
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
// sum_rc' dxp[rc'][cols] (rc' order; x itself if there is no update), chunk
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
        un[u] = (live && col < c1) ? load_raw<T, AL>(A + row * p.ld, col, c1) : zero4;
    }
    __shared__ V s_x[128];
    if (tid < 128) {
        const int64_t c = c0 + tid;
        V xv = (V)0;
        if (c < c1) {
            if (p.upd && cnt > 0) {
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

// ------------------------------------------------------------ launchers --
// Factor `batch` padded matrices (rows x ld each, rows = ld or ld + TB) in
// G: L into Lf, every diagonal tile's inverse into W[bt * P + p].
static hipError_t big_potrf(double *G, double *Lf, int ld, int rows, int batch, double *W,
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
                           (const double *)X, ld, P, t0, L.q, L.rem, h->d_H);
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

template <typename T, typename V>
static hipError_t big_step_typed(const rorbk_handle_s *h, const StepArgs &a, hipStream_t s) {
    const Layout &L = h->L;
    constexpr int RCH = big_rch<T>();
    const double *y = nullptr;
    if (a.ymode == 0) {
        const unsigned g16 = (unsigned)((L.bmax + 15) / 16);
        hipLaunchKernelGGL(k_big_r<V>, dim3(g16), dim3(256), 0, s, h->d_tau, a.cur.tau_index,
                           L.q, L.rem, (const V *)a.b, a.Pin, (int)L.nch_u, (int)L.bmax,
                           h->d_bigr, (const Ctrl *)h->d_ctrl);
        hipLaunchKernelGGL(k_big_y<V>, dim3(g16), dim3(256), 0, s, (const double *)h->d_H,
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
    p.upd = (a.ymode != 2) ? 1 : 0;
    p.y = y;
    p.x = a.x;
    p.xold = h->d_xold;
    p.dxp = h->d_dxp;
    p.gb = (a.ymode == 1) ? a.gb : nullptr;   // fixed blocks update gb in k_big_y
    p.nxt = a.nxt;
    p.Pout = a.Pout;
    p.bmax = (int)L.bmax;
    p.ctrl = h->d_ctrl;
    const unsigned nrc = (unsigned)((L.bmax + RCH - 1) / RCH);
    if (p.upd) {
        if (a.aligned)
            hipLaunchKernelGGL((k_big_upd<T, V, true>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
        else
            hipLaunchKernelGGL((k_big_upd<T, V, false>), dim3(L.nch_u, nrc), dim3(BIG_T), 0, s, p);
    }
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
