// Learned scheduler: per-pair features, a 3-layer MLP (hidden 64, ReLU)
// trained on the GPU with hand-written forward/backward/Adam kernels, and
// BF16 inference that sets each pair's SMM depth l_b and AMC batch count tau.
//
// The estimator itself is untouched: any (l_b in [0, l], tau >= 1) keeps the
// guarantee of Theorem 3.2 / Section 4.2 (the AMC stop rule, eta*, delta and
// l are always the method's own), so the model only moves work between the
// SMM and AMC phases.  Pairs whose predicted error exceeds eps, or whose
// features fall outside the training range, fall back to the greedy switch
// of Eq. (smm-amc).
#include <cmath>
#include <cstdio>
#include <cstring>

#include "geer_internal.h"

namespace geer {

constexpr int kF = GEER_MLP_FEATURES;  // input features
constexpr int kH = GEER_MLP_HIDDEN;    // hidden width
constexpr int kO = GEER_MLP_OUTPUTS;   // outputs: l_b, tau, log10 error
constexpr int kP = kF * kH + kH + kH * kH + kH + kH * kO + kO;  // parameter count

// parameter layout (row-major [in][out])
constexpr int oW1 = 0, oB1 = oW1 + kF * kH, oW2 = oB1 + kH, oB2 = oW2 + kH * kH,
              oW3 = oB2 + kH, oB3 = oW3 + kH * kO;

// ---------------------------------------------------------------------------
// features (one wavefront per pair)
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool sorted_contains(const int32_t *__restrict__ a, int32_t n, int32_t x)
{
    int32_t lo = 0, hi = n;
    while (lo < hi) {
        int32_t mid = (lo + hi) >> 1;
        if (a[mid] < x) lo = mid + 1;
        else hi = mid;
    }
    return lo < n && a[lo] == x;
}

__global__ __launch_bounds__(256) void k_features(
    int64_t nq, const int32_t *__restrict__ s_arr, const int32_t *__restrict__ t_arr,
    const double *__restrict__ eps_arr, const int32_t *__restrict__ ell_arr,
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const int64_t *__restrict__ nbr_work, const int32_t *__restrict__ min_nbr_deg,
    const int32_t *__restrict__ nbr_deg2, double lambda, double log_mean_deg, double rho2,
    double rhod, float *__restrict__ feat)
{
    const int lane = threadIdx.x & 63;
    const int64_t i = (int64_t)blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nq) return;
    const int32_t s = s_arr[i], t = t_arr[i];
    const int32_t bs = row_ptr[s], ds = row_ptr[s + 1] - bs;
    const int32_t bt = row_ptr[t], dt = row_ptr[t + 1] - bt;
    // common neighbours: look up the shorter list in the longer one
    const int32_t *sa = col_idx + (ds <= dt ? bs : bt);
    const int32_t *la = col_idx + (ds <= dt ? bt : bs);
    const int32_t ns = min(ds, dt), nl = max(ds, dt);
    int cn = 0;
    bool edge = false;
    for (int32_t k = lane; k < ns; k += 64) cn += sorted_contains(la, nl, sa[k]) ? 1 : 0;
    for (int32_t k = lane; k < ds; k += 64) edge |= col_idx[bs + k] == t;
    for (int o = 32; o > 0; o >>= 1) {
        cn += __shfl_xor(cn, o);
        edge |= __shfl_xor((int)edge, o) != 0;
    }
    if (lane != 0) return;
    float *f = feat + i * kF;
    f[0] = (float)log2((double)ds);
    f[1] = (float)log2((double)dt);
    f[2] = (float)(ell_arr[i] / 16.0);
    f[3] = (float)log2(1.0 + (double)nbr_work[s]);
    f[4] = (float)log2(1.0 + (double)nbr_work[t]);
    f[5] = (float)log2((double)min_nbr_deg[s]);
    f[6] = (float)log2((double)min_nbr_deg[t]);
    f[7] = edge ? 1.f : 0.f;
    f[8] = (float)log2(1.0 + cn);
    f[9] = (float)log2(1.0 / (1.0 - lambda));
    f[10] = (float)log2(eps_arr[i]);
    f[11] = (float)log2(rho2);
    f[12] = (float)log2(rhod);
    // psi of Eq. (Delta-st) after one product, relative to eps: the hop-1
    // vector of s is 1/d(v) on N(s), so its largest entry is 1/(smallest
    // neighbour degree) and its second largest 1/(second smallest), 0 when
    // d(s) = 1; the first AMC batch at l_b = 1 grows as (psi_1 / eps)^2
    const int32_t lf = ell_arr[i] - 1;
    double psi1 = 0.0;
    if (lf > 0) {
        const int32_t s2 = nbr_deg2[s], t2 = nbr_deg2[t];
        psi1 = psi_of(lf, 1.0 / min_nbr_deg[s], s2 > 0 ? 1.0 / s2 : 0.0, 1.0 / min_nbr_deg[t],
                      t2 > 0 ? 1.0 / t2 : 0.0, 1.0 / ds, 1.0 / dt);
    }
    f[13] = (float)log2(fmax(psi1, ldexp(1.0, -40)) / eps_arr[i]);
    (void)log_mean_deg;
}

// ---------------------------------------------------------------------------
// MLP forward (FP32 master weights or BF16 copy)
// ---------------------------------------------------------------------------

__device__ __forceinline__ float bf16_to_f32(uint16_t h)
{
    return __uint_as_float((uint32_t)h << 16);
}

// round to nearest even
__host__ __device__ inline uint16_t f32_to_bf16(float x)
{
    uint32_t u;
    std::memcpy(&u, &x, 4);
    if ((u & 0x7f800000u) == 0x7f800000u) return (uint16_t)(u >> 16);  // inf / nan
    u += 0x7fffu + ((u >> 16) & 1u);
    return (uint16_t)(u >> 16);
}

template <bool BF16>
__device__ void mlp_eval(const float *__restrict__ pf, const uint16_t *__restrict__ pb,
                         const float *x, float *out)
{
    auto P = [&](int k) -> float { return BF16 ? bf16_to_f32(pb[k]) : pf[k]; };
    float h1[kH], h2[kH];
    for (int k = 0; k < kH; ++k) {
        float a = P(oB1 + k);
        for (int f = 0; f < kF; ++f) a += P(oW1 + f * kH + k) * x[f];
        h1[k] = a > 0.f ? a : 0.f;
    }
    for (int k = 0; k < kH; ++k) {
        float a = P(oB2 + k);
        for (int i = 0; i < kH; ++i) a += P(oW2 + i * kH + k) * h1[i];
        h2[k] = a > 0.f ? a : 0.f;
    }
    for (int o = 0; o < kO; ++o) {
        float a = P(oB3 + o);
        for (int i = 0; i < kH; ++i) a += P(oW3 + i * kO + o) * h2[i];
        out[o] = a;
    }
}

__global__ void k_mlp_forward(int64_t nb, const float *__restrict__ x, const float *__restrict__ pf,
                              const uint16_t *__restrict__ pb, int use_bf16, float *__restrict__ y)
{
    const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nb) return;
    float xin[kF], o[kO];
    for (int f = 0; f < kF; ++f) xin[f] = x[i * kF + f];
    if (use_bf16) mlp_eval<true>(pf, pb, xin, o);
    else mlp_eval<false>(pf, pb, xin, o);
    for (int k = 0; k < kO; ++k) y[i * kO + k] = o[k];
}

// ---------------------------------------------------------------------------
// training: one workgroup; parameters, Adam moments and the gradient stay in
// LDS for all steps.  Every parameter is owned by one thread, which adds the
// samples of a minibatch in a fixed order, so training is deterministic.
// Inputs are normalised features; loss per sample: sum_o w_o (y_hat_o - y_o)^2,
// averaged over the minibatch.  Adam with bias correction.
// ---------------------------------------------------------------------------

constexpr int kTB = 64;  // minibatch capacity

__global__ __launch_bounds__(256) void k_mlp_train(
    float *__restrict__ params, float *__restrict__ adam_m, float *__restrict__ adam_v,
    const float *__restrict__ X, const float *__restrict__ Y, const float *__restrict__ Wt,
    const int64_t *__restrict__ order, int64_t n, int32_t steps, int32_t B, float lr,
    float beta1, float beta2, float adam_eps, int64_t step0, uint64_t seed,
    float *__restrict__ loss_out)
{
    __shared__ float sp[kP], sm[kP], sv[kP], sg[kP];
    __shared__ float sx[kTB][kF];
    __shared__ float sh1[kTB][kH], sh2[kTB][kH], sd1[kTB][kH], sd2[kTB][kH];
    __shared__ float sdo[kTB][kO];
    __shared__ int64_t sidx[kTB];
    __shared__ float sloss[kTB];
    const int tid = threadIdx.x;
    for (int k = tid; k < kP; k += 256) {
        sp[k] = params[k];
        sm[k] = adam_m[k];
        sv[k] = adam_v[k];
    }
    __syncthreads();
    for (int32_t st = 0; st < steps; ++st) {
        const int64_t step = step0 + st + 1;
        if (tid < B) {
            int64_t idx;
            if (order) {
                idx = order[(int64_t)st * B + tid];
            } else {
                // splitmix64 finaliser of (seed, step, slot): uniform with replacement
                uint64_t z = seed + (uint64_t)step * 0x9E3779B97F4A7C15ull + (uint64_t)tid * 0xD1B54A32D192ED03ull;
                z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ull;
                z = (z ^ (z >> 27)) * 0x94D049BB133111EBull;
                z ^= z >> 31;
                idx = (int64_t)(z % (uint64_t)n);
            }
            sidx[tid] = idx;
        }
        __syncthreads();
        for (int e = tid; e < B * kF; e += 256) sx[e / kF][e % kF] = X[sidx[e / kF] * kF + e % kF];
        __syncthreads();
        for (int e = tid; e < B * kH; e += 256) {
            const int b = e / kH, k = e % kH;
            float a = sp[oB1 + k];
            for (int f = 0; f < kF; ++f) a += sp[oW1 + f * kH + k] * sx[b][f];
            sh1[b][k] = a > 0.f ? a : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < B * kH; e += 256) {
            const int b = e / kH, k = e % kH;
            float a = sp[oB2 + k];
            for (int i = 0; i < kH; ++i) a += sp[oW2 + i * kH + k] * sh1[b][i];
            sh2[b][k] = a > 0.f ? a : 0.f;
        }
        __syncthreads();
        if (tid < B) {
            const int b = tid;
            float l = 0.f;
            for (int o = 0; o < kO; ++o) {
                float a = sp[oB3 + o];
                for (int i = 0; i < kH; ++i) a += sp[oW3 + i * kO + o] * sh2[b][i];
                const float diff = a - Y[sidx[b] * kO + o];
                const float w = Wt[sidx[b] * kO + o];
                l += w * diff * diff;
                sdo[b][o] = 2.f * w * diff / (float)B;
            }
            sloss[b] = l;
        }
        __syncthreads();
        for (int e = tid; e < B * kH; e += 256) {
            const int b = e / kH, k = e % kH;
            float a = 0.f;
            for (int o = 0; o < kO; ++o) a += sp[oW3 + k * kO + o] * sdo[b][o];
            sd2[b][k] = sh2[b][k] > 0.f ? a : 0.f;
        }
        __syncthreads();
        for (int e = tid; e < B * kH; e += 256) {
            const int b = e / kH, i = e % kH;
            float a = 0.f;
            for (int k = 0; k < kH; ++k) a += sp[oW2 + i * kH + k] * sd2[b][k];
            sd1[b][i] = sh1[b][i] > 0.f ? a : 0.f;
        }
        __syncthreads();
        for (int k = tid; k < kP; k += 256) {
            float gk = 0.f;
            if (k < oB1) {
                const int f = k / kH, j = k % kH;
                for (int b = 0; b < B; ++b) gk += sx[b][f] * sd1[b][j];
            } else if (k < oW2) {
                const int j = k - oB1;
                for (int b = 0; b < B; ++b) gk += sd1[b][j];
            } else if (k < oB2) {
                const int i = (k - oW2) / kH, j = (k - oW2) % kH;
                for (int b = 0; b < B; ++b) gk += sh1[b][i] * sd2[b][j];
            } else if (k < oW3) {
                const int j = k - oB2;
                for (int b = 0; b < B; ++b) gk += sd2[b][j];
            } else if (k < oB3) {
                const int i = (k - oW3) / kO, o = (k - oW3) % kO;
                for (int b = 0; b < B; ++b) gk += sh2[b][i] * sdo[b][o];
            } else {
                const int o = k - oB3;
                for (int b = 0; b < B; ++b) gk += sdo[b][o];
            }
            sg[k] = gk;
        }
        __syncthreads();
        const float bc1 = 1.f - powf(beta1, (float)step), bc2 = 1.f - powf(beta2, (float)step);
        for (int k = tid; k < kP; k += 256) {
            const float gk = sg[k];
            sm[k] = beta1 * sm[k] + (1.f - beta1) * gk;
            sv[k] = beta2 * sv[k] + (1.f - beta2) * gk * gk;
            sp[k] -= lr * (sm[k] / bc1) / (sqrtf(sv[k] / bc2) + adam_eps);
        }
        if (tid == 0 && loss_out) {
            float L = 0.f;
            for (int b = 0; b < B; ++b) L += sloss[b];
            loss_out[st] = L / (float)B;
        }
        __syncthreads();
    }
    for (int k = tid; k < kP; k += 256) {
        params[k] = sp[k];
        adam_m[k] = sm[k];
        adam_v[k] = sv[k];
    }
}

// gradient of the minibatch loss at the current parameters (no update), for checks
__global__ __launch_bounds__(256) void k_mlp_grad(const float *__restrict__ params,
                                                  const float *__restrict__ X,
                                                  const float *__restrict__ Y,
                                                  const float *__restrict__ Wt, int32_t B,
                                                  float *__restrict__ grad)
{
    __shared__ float sx[kTB][kF];
    __shared__ float sh1[kTB][kH], sh2[kTB][kH], sd1[kTB][kH], sd2[kTB][kH];
    __shared__ float sdo[kTB][kO];
    const int tid = threadIdx.x;
    const float *sp = params;
    for (int e = tid; e < B * kF; e += 256) sx[e / kF][e % kF] = X[e];
    __syncthreads();
    for (int e = tid; e < B * kH; e += 256) {
        const int b = e / kH, k = e % kH;
        float a = sp[oB1 + k];
        for (int f = 0; f < kF; ++f) a += sp[oW1 + f * kH + k] * sx[b][f];
        sh1[b][k] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < B * kH; e += 256) {
        const int b = e / kH, k = e % kH;
        float a = sp[oB2 + k];
        for (int i = 0; i < kH; ++i) a += sp[oW2 + i * kH + k] * sh1[b][i];
        sh2[b][k] = a > 0.f ? a : 0.f;
    }
    __syncthreads();
    if (tid < B) {
        for (int o = 0; o < kO; ++o) {
            float a = sp[oB3 + o];
            for (int i = 0; i < kH; ++i) a += sp[oW3 + i * kO + o] * sh2[tid][i];
            sdo[tid][o] = 2.f * Wt[tid * kO + o] * (a - Y[tid * kO + o]) / (float)B;
        }
    }
    __syncthreads();
    for (int e = tid; e < B * kH; e += 256) {
        const int b = e / kH, k = e % kH;
        float a = 0.f;
        for (int o = 0; o < kO; ++o) a += sp[oW3 + k * kO + o] * sdo[b][o];
        sd2[b][k] = sh2[b][k] > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int e = tid; e < B * kH; e += 256) {
        const int b = e / kH, i = e % kH;
        float a = 0.f;
        for (int k = 0; k < kH; ++k) a += sp[oW2 + i * kH + k] * sd2[b][k];
        sd1[b][i] = sh1[b][i] > 0.f ? a : 0.f;
    }
    __syncthreads();
    for (int k = tid; k < kP; k += 256) {
        float gk = 0.f;
        if (k < oB1) {
            const int f = k / kH, j = k % kH;
            for (int b = 0; b < B; ++b) gk += sx[b][f] * sd1[b][j];
        } else if (k < oW2) {
            for (int b = 0; b < B; ++b) gk += sd1[b][k - oB1];
        } else if (k < oB2) {
            const int i = (k - oW2) / kH, j = (k - oW2) % kH;
            for (int b = 0; b < B; ++b) gk += sh1[b][i] * sd2[b][j];
        } else if (k < oW3) {
            for (int b = 0; b < B; ++b) gk += sd2[b][k - oB2];
        } else if (k < oB3) {
            const int i = (k - oW3) / kO, o = (k - oW3) % kO;
            for (int b = 0; b < B; ++b) gk += sh2[b][i] * sdo[b][o];
        } else {
            for (int b = 0; b < B; ++b) gk += sdo[b][k - oB3];
        }
        grad[k] = gk;
    }
}

// ---------------------------------------------------------------------------
// learned schedule: features -> normalise -> BF16 MLP -> (l_b, tau) or fallback
// ---------------------------------------------------------------------------

constexpr float kRangePad = 0.1f;  // widening of the training range, as a fraction of its span

__global__ void k_learned_apply(QState qs, int64_t nq, const float *__restrict__ feat,
                                const float *__restrict__ norm, const uint16_t *__restrict__ pb,
                                const int32_t *__restrict__ row_ptr,
                                const int32_t *__restrict__ min_nbr_deg,
                                const int64_t *__restrict__ nbr_work, double rho2, double delta,
                                float zmax, int32_t tau_max)
{
    const int64_t q = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
    if (q >= nq) return;
    if (!qs.active_smm[q] && !qs.active_amc[q]) return;  // s == t, l == 0, invalid
    float x[kF], o[kO];
    bool out_of_range = false;
    for (int f = 0; f < kF; ++f) {
        const float raw = feat[q * kF + f];
        x[f] = (raw - norm[f]) / norm[kF + f];
        // per-pair structural features (0..8) must lie in the range seen in
        // training, widened by a tenth of its span (the model extrapolates
        // badly to hubs far beyond its training graphs; the greedy switch
        // does better there); graph-level ones (lambda, eps, cost ratios) are
        // left to the error head
        if (f <= 8) {
            const float lo = norm[2 * kF + f], hi = norm[3 * kF + f];
            const float pad = kRangePad * (hi - lo);
            if (raw < lo - pad || raw > hi + pad || fabsf(x[f]) > zmax) out_of_range = true;
        }
    }
    mlp_eval<true>(nullptr, pb, x, o);
    const int32_t ell = qs.ell[q];
    const double eps = qs.eps[q];
    const double err = exp10((double)o[2]);
    if (out_of_range || !(err <= eps) || !isfinite(o[0]) || !isfinite(o[1])) {
        qs.fallback[q] = 1;  // greedy switch of Eq. (smm-amc) with the default tau
        return;
    }
    int32_t lb = (int32_t)min((double)ell, max(0.0, rint((double)o[0])));
    const int32_t tau = (int32_t)min((double)tau_max, max(1.0, rint((double)o[1])));
    // Cost guards on the predicted depth (regression outputs near a rounding
    // boundary are occasionally far off, and one such pair can cost more
    // walks than thousands of others):
    //  * hop 1 is one scatter per column, so at least one product is taken;
    //  * stopping after one product is rejected when even the first batch of
    //    walks would cost more than hop 2.  After one product the largest
    //    entry of the s-vector is 1/(smallest degree in N(s)) exactly and the
    //    second largest is >= 0, so psi, eta* and eta_1 below are lower
    //    bounds; hop 2 costs rho2 * (sum of neighbour degrees of s and t)
    //    walk-step equivalents.
    if (ell >= 1 && lb < 1) lb = 1;
    if (lb == 1 && ell >= 2) {
        const int32_t s = qs.s[q], t = qs.t[q];
        const double ids = 1.0 / (row_ptr[s + 1] - row_ptr[s]);
        const double idt = 1.0 / (row_ptr[t + 1] - row_ptr[t]);
        const int32_t lf = ell - 1;
        const double psi_lo = psi_of(lf, 1.0 / min_nbr_deg[s], 0.0, 1.0 / min_nbr_deg[t], 0.0, ids, idt);
        const double first = 2.0 * lf * (double)eta1_of(eta_star_of(psi_lo, eps, tau, delta), tau);
        const double hop2 = rho2 * (double)(nbr_work[s] + nbr_work[t]);
        if (first > hop2) lb = 2;
    }
    qs.fallback[q] = 0;
    qs.tau_q[q] = tau;
    qs.lb_target[q] = lb;
    if (lb == 0) {
        // AMC straight from e_s, e_t with the chosen tau
        const int32_t s = qs.s[q], t = qs.t[q];
        const double ids = 1.0 / (row_ptr[s + 1] - row_ptr[s]);
        const double idt = 1.0 / (row_ptr[t + 1] - row_ptr[t]);
        qs.active_smm[q] = 0;
        qs.lf[q] = ell;
        const double psi = psi_of(ell, 1.0, 0.0, 1.0, 0.0, ids, idt);
        const double es = eta_star_of(psi, eps, tau, delta);
        qs.psi[q] = psi;
        qs.eta_star[q] = es;
        qs.eta1[q] = eta1_of(es, tau);
        qs.active_amc[q] = qs.eta1[q] > 0 ? 1 : 0;
        qs.stop[q] = qs.active_amc[q] ? GEER_STOP_CAP : GEER_STOP_NO_WALKS;
    } else {
        qs.active_smm[q] = 1;
        qs.active_amc[q] = 0;
    }
}

}  // namespace geer

// ---------------------------------------------------------------------------
// host side
// ---------------------------------------------------------------------------

struct geer_model {
    int device = 0;
    int64_t step = 0;
    uint64_t seed = 0;
    float norm[4 * geer::kF];  // mean, stdev, lo, hi of the raw features
    float params[geer::kP], adam_m[geer::kP], adam_v[geer::kP];
    float *d_params = nullptr, *d_m = nullptr, *d_v = nullptr, *d_norm = nullptr;
    uint16_t *d_bf16 = nullptr;
    bool dev_valid = false;
};

namespace geer {

static geer_status model_upload(geer_model *m)
{
    if (m->dev_valid) return GEER_OK;
    if (!m->d_params) {
        GEER_HIP(hipMalloc(&m->d_params, kP * sizeof(float)));
        GEER_HIP(hipMalloc(&m->d_m, kP * sizeof(float)));
        GEER_HIP(hipMalloc(&m->d_v, kP * sizeof(float)));
        GEER_HIP(hipMalloc(&m->d_norm, 4 * kF * sizeof(float)));
        GEER_HIP(hipMalloc(&m->d_bf16, kP * sizeof(uint16_t)));
    }
    uint16_t b16[kP];
    for (int k = 0; k < kP; ++k) b16[k] = f32_to_bf16(m->params[k]);
    GEER_HIP(hipMemcpy(m->d_params, m->params, sizeof(m->params), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(m->d_m, m->adam_m, sizeof(m->adam_m), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(m->d_v, m->adam_v, sizeof(m->adam_v), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(m->d_norm, m->norm, sizeof(m->norm), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(m->d_bf16, b16, sizeof(b16), hipMemcpyHostToDevice));
    m->dev_valid = true;
    return GEER_OK;
}

geer_status launch_learned(geer_graph *g, const QueryCtx &c, const geer_model *mc, float *d_feat,
                           int32_t tau_max, hipStream_t st)
{
    geer_model *m = const_cast<geer_model *>(mc);
    GEER_TRY(model_upload(m));
    int tok = prof_begin(g, st);
    hipLaunchKernelGGL(k_features, dim3((int)((c.nq + 3) / 4)), dim3(256), 0, st, c.nq, c.qs.s,
                       c.qs.t, c.qs.eps, c.qs.ell, g->d_row_ptr, g->d_col_idx, g->d_nbr_work,
                       g->d_min_nbr_deg, g->d_nbr_deg2, c.lambda, std::log2((double)g->nnz / g->n),
                       g->rho2, g->rhod, d_feat);
    prof_end(g, tok, PK_FEATURES, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    tok = prof_begin(g, st);
    hipLaunchKernelGGL(k_learned_apply, dim3((int)((c.nq + 255) / 256)), dim3(256), 0, st, c.qs, c.nq,
                       d_feat, m->d_norm, m->d_bf16, g->d_row_ptr, g->d_min_nbr_deg, g->d_nbr_work,
                       g->rho2, c.delta, 8.0f, tau_max);
    prof_end(g, tok, PK_MLP, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

}  // namespace geer

using namespace geer;

extern "C" {

geer_status geer_model_create(uint64_t seed, geer_model **out)
{
    if (!out) return fail(GEER_E_INVALID_ARG, "out is NULL");
    geer_model *m = new geer_model();
    m->seed = seed;
    (void)hipGetDevice(&m->device);
    // He-uniform initialisation from a splitmix64 stream
    uint64_t z = seed * 0x9E3779B97F4A7C15ull + 1;
    auto uni = [&]() {
        z += 0x9E3779B97F4A7C15ull;
        uint64_t x = z;
        x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
        x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
        x ^= x >> 31;
        return (double)(x >> 11) * (1.0 / 9007199254740992.0) * 2.0 - 1.0;
    };
    for (int k = 0; k < kP; ++k) {
        int fan_in = k < oB1 ? kF : (k < oW2 ? 0 : (k < oB2 ? kH : (k < oW3 ? 0 : (k < oB3 ? kH : 0))));
        m->params[k] = fan_in ? (float)(uni() * std::sqrt(6.0 / fan_in)) : 0.f;
        m->adam_m[k] = m->adam_v[k] = 0.f;
    }
    for (int f = 0; f < kF; ++f) {
        m->norm[f] = 0.f;
        m->norm[kF + f] = 1.f;
        m->norm[2 * kF + f] = -1e30f;
        m->norm[3 * kF + f] = 1e30f;
    }
    *out = m;
    return GEER_OK;
}

void geer_model_free(geer_model *m)
{
    if (!m) return;
    void *ptrs[] = {m->d_params, m->d_m, m->d_v, m->d_norm, m->d_bf16};
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    delete m;
}

static const char kMagic[8] = {'G', 'E', 'E', 'R', 'M', 'L', 'P', '1'};

geer_status geer_model_save(const geer_model *m, const char *path)
{
    if (!m || !path) return fail(GEER_E_INVALID_ARG, "NULL argument");
    FILE *f = std::fopen(path, "wb");
    if (!f) return fail(GEER_E_INVALID_ARG, std::string("cannot open ") + path);
    int32_t dims[3] = {kF, kH, kO};
    bool ok = std::fwrite(kMagic, 1, 8, f) == 8 && std::fwrite(dims, 4, 3, f) == 3 &&
              std::fwrite(&m->step, 8, 1, f) == 1 && std::fwrite(&m->seed, 8, 1, f) == 1 &&
              std::fwrite(m->norm, 4, 4 * kF, f) == (size_t)(4 * kF) &&
              std::fwrite(m->params, 4, kP, f) == (size_t)kP &&
              std::fwrite(m->adam_m, 4, kP, f) == (size_t)kP &&
              std::fwrite(m->adam_v, 4, kP, f) == (size_t)kP;
    ok = (std::fclose(f) == 0) && ok;
    return ok ? GEER_OK : fail(GEER_E_MODEL, "write failed");
}

geer_status geer_model_load(const char *path, geer_model **out)
{
    if (!path || !out) return fail(GEER_E_INVALID_ARG, "NULL argument");
    FILE *f = std::fopen(path, "rb");
    if (!f) return fail(GEER_E_MODEL, std::string("cannot open ") + path);
    char magic[8];
    int32_t dims[3];
    geer_model *m = new geer_model();
    bool ok = std::fread(magic, 1, 8, f) == 8 && std::memcmp(magic, kMagic, 8) == 0 &&
              std::fread(dims, 4, 3, f) == 3 && dims[0] == kF && dims[1] == kH && dims[2] == kO &&
              std::fread(&m->step, 8, 1, f) == 1 && std::fread(&m->seed, 8, 1, f) == 1 &&
              std::fread(m->norm, 4, 4 * kF, f) == (size_t)(4 * kF) &&
              std::fread(m->params, 4, kP, f) == (size_t)kP &&
              std::fread(m->adam_m, 4, kP, f) == (size_t)kP &&
              std::fread(m->adam_v, 4, kP, f) == (size_t)kP;
    std::fclose(f);
    if (!ok) {
        delete m;
        return fail(GEER_E_MODEL, std::string("malformed model file ") + path);
    }
    for (int k = 0; k < kP; ++k)
        if (!std::isfinite(m->params[k])) {
            delete m;
            return fail(GEER_E_MODEL, "model has non-finite parameters");
        }
    (void)hipGetDevice(&m->device);
    *out = m;
    return GEER_OK;
}

geer_status geer_model_get_params(const geer_model *m, float *out, int64_t count)
{
    if (!m || !out) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (count != kP) return fail(GEER_E_INVALID_ARG, "count must be GEER_MLP_PARAMS");
    std::memcpy(out, m->params, sizeof(m->params));
    return GEER_OK;
}

geer_status geer_model_set_params(geer_model *m, const float *in, int64_t count)
{
    if (!m || !in) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (count != kP) return fail(GEER_E_INVALID_ARG, "count must be GEER_MLP_PARAMS");
    std::memcpy(m->params, in, sizeof(m->params));
    std::memset(m->adam_m, 0, sizeof(m->adam_m));
    std::memset(m->adam_v, 0, sizeof(m->adam_v));
    m->step = 0;
    m->dev_valid = false;
    return GEER_OK;
}

geer_status geer_model_set_norm(geer_model *m, const float *mean, const float *stdev,
                                const float *lo, const float *hi)
{
    if (!m || !mean || !stdev || !lo || !hi) return fail(GEER_E_INVALID_ARG, "NULL argument");
    for (int f = 0; f < kF; ++f) {
        if (!(stdev[f] > 0.f)) return fail(GEER_E_INVALID_ARG, "stdev must be > 0");
        m->norm[f] = mean[f];
        m->norm[kF + f] = stdev[f];
        m->norm[2 * kF + f] = lo[f];
        m->norm[3 * kF + f] = hi[f];
    }
    m->dev_valid = false;
    return GEER_OK;
}

geer_status geer_graph_set_costs(geer_graph *g, double rho2, double rhod)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (!(rho2 > 0.0) || !(rhod > 0.0) || std::isinf(rho2) || std::isinf(rhod))
        return fail(GEER_E_INVALID_ARG, "cost ratios must be > 0 and finite");
    // Timed ratios vary by a few percent from run to run; the stored values
    // are rounded to the nearest power of 2^(1/2), so that the schedule (and
    // every answer) stays the same unless a ratio moves across a grid
    // boundary.  A ratio within 8% (2^(1/8)) of a grid point always maps to it.
    auto snap = [](double r) { return std::exp2(0.5 * std::nearbyint(2.0 * std::log2(r))); };
    g->rho2 = snap(rho2);
    g->rhod = snap(rhod);
    return GEER_OK;
}

geer_status geer_features(geer_graph *g, int64_t nq, const int32_t *s, const int32_t *t,
                          const double *eps, float *feat_out)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (nq < 0) return fail(GEER_E_INVALID_ARG, "nq must be >= 0");
    if (nq == 0) return GEER_OK;
    if (!s || !t || !eps || !feat_out) return fail(GEER_E_INVALID_ARG, "NULL array");
    if (!g->has_lambda) return fail(GEER_E_NO_LAMBDA, "lambda has not been set");
    for (int64_t i = 0; i < nq; ++i)
        if (s[i] < 0 || s[i] >= g->n || t[i] < 0 || t[i] >= g->n || !(eps[i] > 0.0))
            return fail(GEER_E_INVALID_ARG, "query " + std::to_string(i) + " invalid");
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    std::vector<int32_t> ell(nq);
    for (int64_t i = 0; i < nq; ++i)
        ell[i] = ell_of(g->h_row_ptr[s[i] + 1] - g->h_row_ptr[s[i]], g->h_row_ptr[t[i] + 1] - g->h_row_ptr[t[i]],
                        eps[i], g->lambda);
    DevBuf buf;
    const size_t bytes = (size_t)nq * (2 * sizeof(int32_t) + sizeof(double) + sizeof(int32_t) + kF * sizeof(float));
    GEER_TRY(buf.reserve(bytes));
    double *d_eps = buf.as<double>();
    int32_t *d_s = reinterpret_cast<int32_t *>(d_eps + nq);
    int32_t *d_t = d_s + nq, *d_ell = d_t + nq;
    float *d_f = reinterpret_cast<float *>(d_ell + nq);
    GEER_HIP(hipMemcpyAsync(d_eps, eps, nq * sizeof(double), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_s, s, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_t, t, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_ell, ell.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_features, dim3((int)((nq + 3) / 4)), dim3(256), 0, st, nq, d_s, d_t, d_eps,
                       d_ell, g->d_row_ptr, g->d_col_idx, g->d_nbr_work, g->d_min_nbr_deg,
                       g->d_nbr_deg2, g->lambda, std::log2((double)g->nnz / g->n), g->rho2, g->rhod,
                       d_f);
    GEER_HIP(hipGetLastError());
    GEER_HIP(hipMemcpyAsync(feat_out, d_f, (size_t)nq * kF * sizeof(float), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    buf.release();
    return GEER_OK;
}

geer_status geer_mlp_forward(geer_model *m, int64_t nb, const float *x, int32_t use_bf16, float *y_out)
{
    if (!m || (nb > 0 && (!x || !y_out))) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (nb <= 0) return nb == 0 ? GEER_OK : fail(GEER_E_INVALID_ARG, "nb must be >= 0");
    GEER_TRY(model_upload(m));
    DevBuf buf;
    GEER_TRY(buf.reserve((size_t)nb * (kF + kO) * sizeof(float)));
    float *d_x = buf.as<float>(), *d_y = d_x + (size_t)nb * kF;
    GEER_HIP(hipMemcpy(d_x, x, (size_t)nb * kF * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_mlp_forward, dim3((int)((nb + 127) / 128)), dim3(128), 0, 0, nb, d_x, m->d_params,
                       m->d_bf16, use_bf16 ? 1 : 0, d_y);
    GEER_HIP(hipGetLastError());
    GEER_HIP(hipMemcpy(y_out, d_y, (size_t)nb * kO * sizeof(float), hipMemcpyDeviceToHost));
    buf.release();
    return GEER_OK;
}

geer_status geer_mlp_grad(geer_model *m, int32_t nb, const float *x, const float *y, const float *w,
                          float *grad_out)
{
    if (!m || !x || !y || !w || !grad_out) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (nb < 1 || nb > kTB) return fail(GEER_E_INVALID_ARG, "nb must be in 1..64");
    GEER_TRY(model_upload(m));
    DevBuf buf;
    GEER_TRY(buf.reserve(((size_t)nb * (kF + 2 * kO) + kP) * sizeof(float)));
    float *d_x = buf.as<float>(), *d_y = d_x + (size_t)nb * kF, *d_w = d_y + (size_t)nb * kO,
          *d_g = d_w + (size_t)nb * kO;
    GEER_HIP(hipMemcpy(d_x, x, (size_t)nb * kF * sizeof(float), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(d_y, y, (size_t)nb * kO * sizeof(float), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(d_w, w, (size_t)nb * kO * sizeof(float), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_mlp_grad, dim3(1), dim3(256), 0, 0, m->d_params, d_x, d_y, d_w, nb, d_g);
    GEER_HIP(hipGetLastError());
    GEER_HIP(hipMemcpy(grad_out, d_g, kP * sizeof(float), hipMemcpyDeviceToHost));
    buf.release();
    return GEER_OK;
}

geer_status geer_mlp_train(geer_model *m, int64_t n, const float *x, const float *y, const float *w,
                           int32_t steps, int32_t batch, double lr, const int64_t *order,
                           float *loss_out)
{
    if (!m || !x || !y || !w) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (n < 1 || steps < 0 || batch < 1 || batch > kTB || !(lr > 0.0))
        return fail(GEER_E_INVALID_ARG, "bad training arguments (batch must be 1..64)");
    if (steps == 0) return GEER_OK;
    if (order)
        for (int64_t i = 0; i < (int64_t)steps * batch; ++i)
            if (order[i] < 0 || order[i] >= n) return fail(GEER_E_INVALID_ARG, "order index out of range");
    GEER_TRY(model_upload(m));
    DevBuf buf;
    const size_t bytes = (size_t)n * (kF + 2 * kO) * sizeof(float) + (size_t)steps * sizeof(float) +
                         (order ? (size_t)steps * batch * sizeof(int64_t) : 0) + 64;
    GEER_TRY(buf.reserve(bytes));
    float *d_x = buf.as<float>(), *d_y = d_x + (size_t)n * kF, *d_w = d_y + (size_t)n * kO,
          *d_l = d_w + (size_t)n * kO;
    int64_t *d_o = order ? reinterpret_cast<int64_t *>(
                               (char *)buf.ptr + (((char *)(d_l + steps) - (char *)buf.ptr + 7) / 8) * 8)
                         : nullptr;
    GEER_HIP(hipMemcpy(d_x, x, (size_t)n * kF * sizeof(float), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(d_y, y, (size_t)n * kO * sizeof(float), hipMemcpyHostToDevice));
    GEER_HIP(hipMemcpy(d_w, w, (size_t)n * kO * sizeof(float), hipMemcpyHostToDevice));
    if (order) GEER_HIP(hipMemcpy(d_o, order, (size_t)steps * batch * sizeof(int64_t), hipMemcpyHostToDevice));
    hipLaunchKernelGGL(k_mlp_train, dim3(1), dim3(256), 0, 0, m->d_params, m->d_m, m->d_v, d_x, d_y, d_w,
                       d_o, n, steps, batch, (float)lr, 0.9f, 0.999f, 1e-8f, m->step, m->seed, d_l);
    GEER_HIP(hipGetLastError());
    GEER_HIP(hipDeviceSynchronize());
    GEER_HIP(hipMemcpy(m->params, m->d_params, sizeof(m->params), hipMemcpyDeviceToHost));
    GEER_HIP(hipMemcpy(m->adam_m, m->d_m, sizeof(m->adam_m), hipMemcpyDeviceToHost));
    GEER_HIP(hipMemcpy(m->adam_v, m->d_v, sizeof(m->adam_v), hipMemcpyDeviceToHost));
    if (loss_out) GEER_HIP(hipMemcpy(loss_out, d_l, (size_t)steps * sizeof(float), hipMemcpyDeviceToHost));
    m->step += steps;
    // refresh the BF16 inference copy
    uint16_t b16[kP];
    for (int k = 0; k < kP; ++k) b16[k] = f32_to_bf16(m->params[k]);
    GEER_HIP(hipMemcpy(m->d_bf16, b16, sizeof(b16), hipMemcpyHostToDevice));
    buf.release();
    return GEER_OK;
}

}  // extern "C"
