// k_gmres.hip -- the outer loop of flexible AB-GMRES with ROR-BK inner
// iterations (appendix, Algorithm 3): start vector, modified Gram-Schmidt,
// Givens rotations of the Hessenberg least-squares problem, and the final
// update x += Z y.  The inner iterations are the ROR-BK kernels themselves.
// Every reduction has a fixed order.
#include "rorbk_device.h"

namespace rorbk {

constexpr int GM_T = 1024;   // threads of the single-workgroup kernels

// r0 = b - sum_seg axp[seg] (axp = A x0), beta = ||r0||, v_1 = r0 / beta,
// g[0] = beta.  out[0] = beta.
__global__ __launch_bounds__(GM_T) void k_gmres_start(const double *__restrict__ b,
                                                      const double *__restrict__ axp, int nseg,
                                                      int64_t m, double *__restrict__ v1,
                                                      double *__restrict__ g,
                                                      double *__restrict__ out) {
    __shared__ double sh[16];
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += GM_T) {
        double ax = 0.0;
        for (int sg = 0; sg < nseg; ++sg) ax += axp[(int64_t)sg * m + i];
        const double r = b[i] - ax;
        v1[i] = r;
        s = __builtin_fma(r, r, s);
    }
    s = block_sum(s, sh);
    const double beta = sqrt(s);
    if (beta > 0.0)
        for (int64_t i = threadIdx.x; i < m; i += GM_T) v1[i] = v1[i] / beta;
    if (threadIdx.x == 0) {
        g[0] = beta;
        out[0] = beta;
    }
}

// w = A z_k (from the segment products) orthogonalised against v_1..v_{k+1}
// (0-based columns 0..k of V) by modified Gram-Schmidt: h_i = <w, v_i>,
// w -= h_i v_i in order; then h_{k+1} = ||w|| and column k+1 of V = w / ||w||.
// hcol receives h_0..h_{k+1}.
// The same modified Gram-Schmidt over many workgroups, one launch per phase
// (a phase needs the previous one's complete inner product).  Workgroup b owns
// the contiguous rows [b * per, (b + 1) * per); each phase first forms the
// previous coefficient from the previous phase's MG_WG partial sums (added in
// workgroup order, the same value in every workgroup), then makes one pass
// over its rows:
//   phase 0:           w = sum_seg axp;           partial <w, v_0>
//   phase j in 1..k:   w -= h_{j-1} v_{j-1};      partial <w, v_j>
//   phase k + 1:       w -= h_k v_k;               partial <w, w>
//   phase k + 2:       h_{k+1} = sqrt(sum);        w /= h_{k+1} (if positive)
// Thread t of a workgroup sums its rows t, t + MG_T, ... in order; the
// workgroup sum has a fixed order (block_sum).  part holds two alternating
// sets of MG_WG partials; workgroup 0 writes hcol.
constexpr int MG_WG = 128, MG_T = 256;

__global__ __launch_bounds__(MG_T) void k_gmres_mgs_phase(double *__restrict__ V, int64_t m, int k,
                                                          int j, const double *__restrict__ axp,
                                                          int nseg, double *__restrict__ part,
                                                          double *__restrict__ hcol) {
    __shared__ double sh[16];
    __shared__ double s_h;
    double *w = V + (int64_t)(k + 1) * m;
    const int64_t per = (m + MG_WG - 1) / MG_WG;
    const int64_t r0 = (int64_t)blockIdx.x * per;
    const int64_t r1 = (r0 + per < m) ? r0 + per : m;
    // the previous phase's coefficient
    if (j > 0) {
        if (threadIdx.x < 64) {
            const double *pp = part + ((j - 1) & 1) * MG_WG;
            double a = 0.0;
            for (int q = threadIdx.x; q < MG_WG; q += 64) a += pp[q];
#pragma unroll
            for (int off = 32; off >= 1; off >>= 1) a += __shfl_xor(a, off, 64);
            if (threadIdx.x == 0) {
                const double hv = (j == k + 2) ? sqrt(a) : a;
                s_h = hv;
                if (blockIdx.x == 0) hcol[j - 1] = hv;
            }
        }
        __syncthreads();
    }
    const double hp = (j > 0) ? s_h : 0.0;
    if (j == k + 2) {
        if (hp > 0.0)
            for (int64_t i = r0 + threadIdx.x; i < r1; i += MG_T) w[i] = w[i] / hp;
        return;
    }
    const double *vp = V + (int64_t)(j > 0 ? j - 1 : 0) * m;
    const double *vj = (j <= k) ? V + (int64_t)j * m : w;
    double sacc = 0.0;
    for (int64_t i = r0 + threadIdx.x; i < r1; i += MG_T) {
        double wi;
        if (j == 0) {
            wi = 0.0;
            for (int sg = 0; sg < nseg; ++sg) wi += axp[(int64_t)sg * m + i];
        } else {
            wi = __builtin_fma(-hp, vp[i], w[i]);
        }
        w[i] = wi;
        const double v = (j <= k) ? vj[i] : wi;
        sacc = __builtin_fma(wi, v, sacc);
    }
    sacc = block_sum(sacc, sh);
    if (threadIdx.x == 0) part[(j & 1) * MG_WG + blockIdx.x] = sacc;
}

// Column k of the Hessenberg matrix into R (column-major, ld M1), the earlier
// rotations applied to it, a new rotation zeroing h_{k+1,k}, and g updated.
// est[0] = |g_{k+1}| (the residual norm of the least-squares problem),
// est[1] = h_{k+1,k}.
__global__ void k_gmres_givens(const double *__restrict__ hcol, int k, int M1,
                               double *__restrict__ R, double *__restrict__ cs,
                               double *__restrict__ sn, double *__restrict__ g,
                               double *__restrict__ est) {
    if (threadIdx.x != 0) return;
    double *col = R + (int64_t)k * M1;
    for (int i = 0; i <= k + 1; ++i) col[i] = hcol[i];
    for (int i = 0; i < k; ++i) {
        const double a = col[i], c = col[i + 1];
        col[i] = cs[i] * a + sn[i] * c;
        col[i + 1] = -sn[i] * a + cs[i] * c;
    }
    const double a = col[k], c = col[k + 1];
    const double d = sqrt(a * a + c * c);
    cs[k] = (d > 0.0) ? a / d : 1.0;
    sn[k] = (d > 0.0) ? c / d : 0.0;
    col[k] = d;
    col[k + 1] = 0.0;
    g[k + 1] = -sn[k] * g[k];
    g[k] = cs[k] * g[k];
    est[0] = fabs(g[k + 1]);
    est[1] = hcol[k + 1];
}

// y = R^{-1} g over the first kend columns (every workgroup solves the small
// triangle itself), then x_j += sum_k y_k Z[k][j] in k order.
__global__ __launch_bounds__(256) void k_gmres_update(const double *__restrict__ Z, int64_t n,
                                                      const double *__restrict__ R,
                                                      const double *__restrict__ g, int kend,
                                                      int M1, double *__restrict__ x) {
    extern __shared__ double yv[];
    if (threadIdx.x == 0) {
        for (int i = kend - 1; i >= 0; --i) {
            double s = g[i];
            for (int j = i + 1; j < kend; ++j) s -= R[(int64_t)j * M1 + i] * yv[j];
            yv[i] = s / R[(int64_t)i * M1 + i];
        }
    }
    __syncthreads();
    const int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (c >= n) return;
    double s = x[c];
    for (int j = 0; j < kend; ++j) s = __builtin_fma(yv[j], Z[(int64_t)j * n + c], s);
    x[c] = s;
}

hipError_t launch_gmres_start(const double *b, const double *axp, int nseg, int64_t m,
                              double *v1, double *g, double *out, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_start, dim3(1), dim3(GM_T), 0, s, b, axp, nseg, m, v1, g, out);
    return hipGetLastError();
}

hipError_t launch_gmres_step(double *V, int64_t m, int k, const double *axp, int nseg,
                             double *hcol, int M1, double *R, double *cs, double *sn, double *g,
                             double *est, double *part, hipStream_t s) {
    for (int j = 0; j <= k + 2; ++j)
        hipLaunchKernelGGL(k_gmres_mgs_phase, dim3(MG_WG), dim3(MG_T), 0, s, V, m, k, j, axp,
                           nseg, part, hcol);
    hipLaunchKernelGGL(k_gmres_givens, dim3(1), dim3(64), 0, s, (const double *)hcol, k, M1, R,
                       cs, sn, g, est);
    return hipGetLastError();
}

hipError_t launch_gmres_update(const double *Z, int64_t n, const double *R, const double *g,
                               int kend, int M1, double *x, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_update, dim3((unsigned)((n + 255) / 256)), dim3(256),
                       sizeof(double) * (size_t)kend, s, Z, n, R, g, kend, M1, x);
    return hipGetLastError();
}

}  // namespace rorbk
