// lambda = max(|lambda_2|, |lambda_n|) of P = D^-1 A (Theorem 3.1), computed
// once per graph (the paper's preprocessing step, Section 3.1).
//
// P is similar to N = D^-1/2 A D^-1/2, whose top eigenvector sqrt(d) has
// eigenvalue 1.  Lanczos runs on N with that vector deflated and full
// reorthogonalisation, in FP64 on the GPU: the products with N are CSR
// gathers, the projections are batched dot products over the stored basis.
// The small tridiagonal problem is solved on the host (Sturm bisection and
// inverse iteration).  The extreme Ritz values are widened by their residual
// norms beta_m |y_m|, which gives an estimate from above of the extreme
// eigenvalues (Ritz values alone approach them from inside).
#include <algorithm>
#include <cmath>
#include <vector>

#include "geer_internal.h"

namespace geer {

// y(v) = d(v)^-1/2 sum_{u in N(v)} d(u)^-1/2 x(u); one wavefront per row.
__global__ __launch_bounds__(256) void k_norm_spmv(int32_t n, const int32_t *__restrict__ row_ptr,
                                                   const int32_t *__restrict__ col_idx,
                                                   const double *__restrict__ isd,
                                                   const double *__restrict__ xs,
                                                   double *__restrict__ y)
{
    // xs = D^{-1/2} x was formed beforehand, so each CSR entry gathers one value
    const int lane = threadIdx.x & 63;
    for (int64_t v = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6); v < n;
         v += (int64_t)gridDim.x * 4) {
        const int32_t b = row_ptr[v], e = row_ptr[v + 1];
        double acc = 0.0;
        for (int32_t k = b + lane; k < e; k += 64) acc += xs[col_idx[k]];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if (lane == 0) y[v] = isd[v] * acc;
    }
}

__global__ __launch_bounds__(256) void k_mul(int32_t n, const double *__restrict__ a,
                                             const double *__restrict__ x, double *__restrict__ out)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        out[i] = a[i] * x[i];
}

// <V_k, w> for k < m (V stored vector-major, stride n), in two passes with a
// fixed summation order: block b sums its slice of every product into
// part[k * nb + b], then one block per k adds the nb partials.
constexpr int kDotBlocks = 512;

__global__ __launch_bounds__(256) void k_dots_partial(int32_t n, const double *__restrict__ V, int m,
                                                      const double *__restrict__ w,
                                                      double *__restrict__ part)
{
    const int b = blockIdx.x, nb = gridDim.x;
    const int64_t per = ((int64_t)n + nb - 1) / nb;
    const int64_t i0 = (int64_t)b * per, i1 = min((int64_t)n, i0 + per);
    __shared__ double sh[4];
    for (int k = 0; k < m; ++k) {
        const double *vk = V + (size_t)k * n;
        double acc = 0.0;
        for (int64_t i = i0 + threadIdx.x; i < i1; i += blockDim.x) acc += vk[i] * w[i];
        for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
        if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
        __syncthreads();
        if (threadIdx.x == 0) part[(size_t)k * nb + b] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
        __syncthreads();
    }
}

__global__ __launch_bounds__(256) void k_dots_final(int nb, int m, const double *__restrict__ part,
                                                    double *__restrict__ out)
{
    const int k = blockIdx.x;
    if (k >= m) return;
    double acc = 0.0;
    for (int i = threadIdx.x; i < nb; i += blockDim.x) acc += part[(size_t)k * nb + i];
    for (int o = 32; o > 0; o >>= 1) acc += __shfl_xor(acc, o);
    __shared__ double sh[4];
    if ((threadIdx.x & 63) == 0) sh[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) out[k] = (sh[0] + sh[1]) + (sh[2] + sh[3]);
}

// w -= sum_k c[k] V_k, then optionally write w * scale to dst.
__global__ __launch_bounds__(256) void k_subtract(int32_t n, const double *__restrict__ V, int m,
                                                  const double *__restrict__ c,
                                                  double *__restrict__ w)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x) {
        double acc = w[i];
        for (int k = 0; k < m; ++k) acc -= c[k] * V[(size_t)k * n + i];
        w[i] = acc;
    }
}

__global__ __launch_bounds__(256) void k_scale_copy(int32_t n, const double *__restrict__ w,
                                                    double s, double *__restrict__ dst)
{
    for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
         i += (int64_t)gridDim.x * blockDim.x)
        dst[i] = w[i] * s;
}

// ---------------------------------------------------------------------------
// host: symmetric tridiagonal helpers (alpha[0..m-1], beta[0..m-2])
// ---------------------------------------------------------------------------

static int sturm_count_below(const std::vector<double> &a, const std::vector<double> &b, int m,
                             double x)
{
    int cnt = 0;
    double q = a[0] - x;
    if (q < 0) ++cnt;
    for (int i = 1; i < m; ++i) {
        double qq = q == 0.0 ? 1e-300 : q;
        q = (a[i] - x) - b[i - 1] * b[i - 1] / qq;
        if (q < 0) ++cnt;
    }
    return cnt;
}

// k-th smallest eigenvalue (0-based) by bisection.
static double tri_eig(const std::vector<double> &a, const std::vector<double> &b, int m, int k)
{
    double lo = a[0], hi = a[0];
    for (int i = 0; i < m; ++i) {
        double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < m ? std::fabs(b[i]) : 0.0);
        lo = std::min(lo, a[i] - r);
        hi = std::max(hi, a[i] + r);
    }
    for (int it = 0; it < 200; ++it) {
        double mid = 0.5 * (lo + hi);
        if (mid <= lo || mid >= hi) break;
        if (sturm_count_below(a, b, m, mid) > k) hi = mid;
        else lo = mid;
    }
    return 0.5 * (lo + hi);
}

// |last component| of the unit eigenvector of T for eigenvalue theta (inverse iteration).
static double tri_last_component(const std::vector<double> &a, const std::vector<double> &b,
                                 int m, double theta)
{
    if (m == 1) return 1.0;
    std::vector<double> y(m, 1.0), cp(m), dp(m);
    const double shift = theta + 1e-13 * std::max(1.0, std::fabs(theta));
    for (int it = 0; it < 4; ++it) {
        // Thomas algorithm on (T - shift I) z = y
        double den = a[0] - shift;
        if (den == 0.0) den = 1e-300;
        cp[0] = b[0] / den;
        dp[0] = y[0] / den;
        for (int i = 1; i < m; ++i) {
            den = (a[i] - shift) - b[i - 1] * cp[i - 1];
            if (den == 0.0) den = 1e-300;
            cp[i] = i + 1 < m ? b[i] / den : 0.0;
            dp[i] = (y[i] - b[i - 1] * dp[i - 1]) / den;
        }
        y[m - 1] = dp[m - 1];
        for (int i = m - 2; i >= 0; --i) y[i] = dp[i] - cp[i] * y[i + 1];
        double nrm = 0.0;
        for (double v : y) nrm += v * v;
        nrm = std::sqrt(nrm);
        if (!(nrm > 0.0) || !std::isfinite(nrm)) return 1.0;
        for (double &v : y) v /= nrm;
    }
    return std::fabs(y[m - 1]);
}

}  // namespace geer

using namespace geer;

extern "C" geer_status geer_graph_compute_lambda(geer_graph *g, int32_t max_iter, double tol,
                                                 uint64_t seed, double *lambda_out)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (max_iter < 2) return fail(GEER_E_INVALID_ARG, "max_iter must be >= 2");
    if (!(tol > 0.0)) return fail(GEER_E_INVALID_ARG, "tol must be > 0");
    GEER_HIP(hipSetDevice(g->device));
    const int32_t n = g->n;
    const int m_max = std::min<int>(max_iter, n - 1);
    hipStream_t st = g->stream;
    // device memory: basis (u + m_max + 1 vectors), w, isd, coefficient buffer
    DevBuf basis, work;
    GEER_TRY(basis.reserve((size_t)(m_max + 2) * n * sizeof(double)));
    const int nb = std::max(1, std::min(kDotBlocks, (n + 255) / 256));
    GEER_TRY(work.reserve((size_t)3 * n * sizeof(double) + (size_t)(m_max + 2) * sizeof(double) +
                          (size_t)(m_max + 2) * nb * sizeof(double)));
    double *V = basis.as<double>();          // V[0] = u (deflated vector), V[1..] Lanczos basis
    double *w = work.as<double>();
    double *isd = w + n;
    double *coef = isd + n;
    double *part = coef + (m_max + 2);
    double *xs = part + (size_t)(m_max + 2) * nb;  // D^{-1/2} V_j for the product
    std::vector<int32_t> rp(n + 1);
    GEER_HIP(hipMemcpy(rp.data(), g->d_row_ptr, (n + 1) * sizeof(int32_t), hipMemcpyDeviceToHost));
    std::vector<double> h_isd(n), h_u(n), h_v(n);
    double unorm = 0.0, deg_sum = 0.0;
    for (int32_t v = 0; v < n; ++v) {
        double d = rp[v + 1] - rp[v];
        h_isd[v] = 1.0 / std::sqrt(d);
        deg_sum += d;
    }
    unorm = std::sqrt(deg_sum);
    for (int32_t v = 0; v < n; ++v) h_u[v] = std::sqrt((double)(rp[v + 1] - rp[v])) / unorm;
    // start vector: splitmix64 uniforms in (-1/2, 1/2)
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 0x632BE59BD9B4E019ull;
    for (int32_t v = 0; v < n; ++v) {
        z += 0x9E3779B97F4A7C15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        x ^= x >> 31;
        h_v[v] = (double)(x >> 11) * (1.0 / 9007199254740992.0) - 0.5;
    }
    GEER_HIP(hipMemcpy(isd, h_isd.data(), n * sizeof(double), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(V, h_u.data(), n * sizeof(double), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(w, h_v.data(), n * sizeof(double), hipMemcpyHostToDevice));
    const int eb = std::max(1, std::min(g->num_cus * 8, (n + 255) / 256));
    const int sb = std::max(1, std::min(g->num_cus * 8, (n + 3) / 4));
    // coef[k] = <Vp_k, x> for k < m
    auto dots = [&](const double *Vp, int m, const double *x) {
        hipLaunchKernelGGL(k_dots_partial, dim3(nb), dim3(256), 0, st, n, Vp, m, x, part);
        hipLaunchKernelGGL(k_dots_final, dim3(m), dim3(256), 0, st, nb, m, part, coef);
    };
    auto orthonormalise = [&](int nvec, double *beta_out) -> geer_status {
        // two passes of classical Gram-Schmidt against V[0..nvec-1]
        for (int pass = 0; pass < 2; ++pass) {
            dots(V, nvec, w);
            hipLaunchKernelGGL(k_subtract, dim3(eb), dim3(256), 0, st, n, V, nvec, coef, w);
        }
        dots(w, 1, w);
        GEER_HIP(hipGetLastError());
        double nn = 0.0;
        GEER_HIP(hipMemcpyAsync(&nn, coef, sizeof(double), hipMemcpyDeviceToHost, st));
        GEER_HIP(hipStreamSynchronize(st));
        *beta_out = std::sqrt(std::max(nn, 0.0));
        return GEER_OK;
    };
    double beta0 = 0.0;
    GEER_TRY(orthonormalise(1, &beta0));
    if (!(beta0 > 0.0)) return fail(GEER_E_DEVICE, "Lanczos start vector vanished");
    hipLaunchKernelGGL(k_scale_copy, dim3(eb), dim3(256), 0, st, n, w, 1.0 / beta0, V + (size_t)n);
    std::vector<double> alpha, beta;
    double lam_hi = 0.0, lam_lo = 0.0, res_hi = 1.0, res_lo = 1.0;
    int m = 0;
    for (int j = 0; j < m_max; ++j) {
        // w = N V_j, then orthogonalise against u and V_1..V_j (alpha = <V_j, w> first)
        hipLaunchKernelGGL(k_mul, dim3(eb), dim3(256), 0, st, n, isd, V + (size_t)(j + 1) * n, xs);
        hipLaunchKernelGGL(k_norm_spmv, dim3(sb), dim3(256), 0, st, n, g->d_row_ptr, g->d_col_idx,
                           isd, xs, w);
        dots(V + (size_t)(j + 1) * n, 1, w);
        GEER_HIP(hipGetLastError());
        double a = 0.0;
        GEER_HIP(hipMemcpyAsync(&a, coef, sizeof(double), hipMemcpyDeviceToHost, st));
        GEER_HIP(hipStreamSynchronize(st));
        double b = 0.0;
        GEER_TRY(orthonormalise(j + 2, &b));
        alpha.push_back(a);
        m = j + 1;
        const bool last = (j + 1 == m_max) || !(b > 1e-12);
        if (m % 10 == 0 || last) {
            lam_hi = tri_eig(alpha, beta, m, m - 1);
            lam_lo = tri_eig(alpha, beta, m, 0);
            res_hi = b * tri_last_component(alpha, beta, m, lam_hi);
            res_lo = b * tri_last_component(alpha, beta, m, lam_lo);
            if ((res_hi < tol && res_lo < tol) || last) break;
        }
        beta.push_back(b);
        hipLaunchKernelGGL(k_scale_copy, dim3(eb), dim3(256), 0, st, n, w, 1.0 / b, V + (size_t)(j + 2) * n);
        GEER_HIP(hipGetLastError());
    }
    basis.release();
    work.release();
    const double lam = std::max(lam_hi + res_hi, -(lam_lo - res_lo));
    if (!(lam >= 0.0) || !std::isfinite(lam)) return fail(GEER_E_DEVICE, "Lanczos produced no estimate");
    if (lam >= 1.0) return fail(GEER_E_BIPARTITE, "lambda estimate >= 1: graph is (nearly) bipartite");
    GEER_TRY(geer_graph_set_lambda(g, lam));
    if (lambda_out) *lambda_out = lam;
    return GEER_OK;
}
