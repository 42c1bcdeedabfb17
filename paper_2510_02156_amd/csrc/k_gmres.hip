// k_gmres.hip -- the outer loop of flexible AB-GMRES with ROR-BK inner
// iterations (appendix, Algorithm 3): start vector, modified Gram-Schmidt,
// Givens rotations of the Hessenberg least-squares problem, and the final
// update x += Z y.  The inner iterations are the ROR-BK kernels themselves.
// Every reduction runs in one workgroup in a fixed order.
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
// hcol receives h_0..h_{k+1}.  Thread t owns rows t, t + GM_T, ...
__global__ __launch_bounds__(GM_T) void k_gmres_mgs(double *__restrict__ V, int64_t m, int k,
                                                    const double *__restrict__ axp, int nseg,
                                                    double *__restrict__ hcol) {
    __shared__ double sh[16];
    double *w = V + (int64_t)(k + 1) * m;
    for (int64_t i = threadIdx.x; i < m; i += GM_T) {
        double ax = 0.0;
        for (int sg = 0; sg < nseg; ++sg) ax += axp[(int64_t)sg * m + i];
        w[i] = ax;
    }
    for (int j = 0; j <= k; ++j) {
        const double *vj = V + (int64_t)j * m;
        double s = 0.0;
        for (int64_t i = threadIdx.x; i < m; i += GM_T) s = __builtin_fma(w[i], vj[i], s);
        const double h = block_sum(s, sh);
        for (int64_t i = threadIdx.x; i < m; i += GM_T) w[i] = __builtin_fma(-h, vj[i], w[i]);
        if (threadIdx.x == 0) hcol[j] = h;
    }
    double s = 0.0;
    for (int64_t i = threadIdx.x; i < m; i += GM_T) s = __builtin_fma(w[i], w[i], s);
    const double hn = sqrt(block_sum(s, sh));
    if (hn > 0.0)
        for (int64_t i = threadIdx.x; i < m; i += GM_T) w[i] = w[i] / hn;
    if (threadIdx.x == 0) hcol[k + 1] = hn;
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
                             double *est, hipStream_t s) {
    hipLaunchKernelGGL(k_gmres_mgs, dim3(1), dim3(GM_T), 0, s, V, m, k, axp, nseg, hcol);
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
