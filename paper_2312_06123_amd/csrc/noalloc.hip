// Algorithm 1 (AMC) for one pair without any device allocation: every
// scratch buffer of the call lives in one fixed file-scope device array.
//
// For callers that cannot allocate device memory (code under HIP graph
// capture, tight serving loops, harnesses that forbid hipMalloc).  The array
// is GEER_AMC_SCRATCH_BYTES per device; each device the library runs on
// holds its own copy until the process ends.  Host code never passes the
// array's name to a kernel or a copy (on the host that name is a stand-in,
// not a device address): its device address is looked up once per device
// with hipGetSymbolAddress and kept in a table.
#include <cmath>
#include <mutex>

#include "geer_internal.h"

namespace geer {

static __device__ __align__(256) unsigned char scratch[GEER_AMC_SCRATCH_BYTES];

// Layout of the scratch array (byte offsets).
constexpr size_t kScrQState = 0;        // QState arrays of one query
constexpr size_t kScrChunkOff = 4096;   // chunk prefix sums: 2 x int64
constexpr size_t kScrMisc = 4352;       // kMiscWords x int64
constexpr size_t kScrColstat = 4608;    // top-2 of the two columns: m1[kCols], m2[kCols] (FP64)
constexpr size_t kScrR = 6656;          // r' of the finalize pass (FP64)
constexpr size_t kScrBad = 6912;        // invalid-vector flag (uint32)
constexpr size_t kScrZpart = 16384;     // chunk partials (sum Z, sum Z^2) up to the end
constexpr int64_t kScrZpartCap = (int64_t)((GEER_AMC_SCRATCH_BYTES - kScrZpart) / sizeof(double2));
static_assert(kScrChunkOff >= 64 && kScrMisc >= kScrChunkOff + 2 * sizeof(int64_t) &&
                  kScrColstat >= kScrMisc + kMiscWords * sizeof(int64_t) &&
                  kScrR >= kScrColstat + 2 * kCols * sizeof(double) && kScrBad >= kScrR + 8 &&
                  kScrZpart >= kScrBad + 4 && kScrZpartCap > 0,
              "scratch regions overlap");

constexpr int kMaxDevices = 64;
static std::mutex g_scratch_mu;
static unsigned char *g_scratch_ptr[kMaxDevices] = {};

// Device address of this device's scratch array (the device must be current).
static geer_status scratch_on_device(int device, unsigned char **out)
{
    if (device < 0 || device >= kMaxDevices) return fail(GEER_E_DEVICE, "device index out of range");
    std::lock_guard<std::mutex> lk(g_scratch_mu);
    if (!g_scratch_ptr[device]) {
        void *p = nullptr;
        const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
        if (e != hipSuccess || !p)
            return fail(GEER_E_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
        g_scratch_ptr[device] = static_cast<unsigned char *>(p);
    }
    *out = g_scratch_ptr[device];
    return GEER_OK;
}

__global__ void k_clear_flag(uint32_t *flag) { *flag = 0u; }

// Flag vectors that are negative, NaN or infinite (the walk sum assumes
// finite non-negative entries).
template <class T>
__global__ __launch_bounds__(256) void k_check_vectors(const T *__restrict__ xy, int64_t count,
                                                       uint32_t *__restrict__ bad)
{
    bool any = false;
    for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count;
         i += (int64_t)gridDim.x * blockDim.x) {
        const T v = xy[i];
        any |= !(v >= T(0)) || isinf(v);
    }
    if (__any(any) && (threadIdx.x & 63) == 0) atomicOr(bad, 1u);
}

__global__ void k_amc_result(QState qs, double *__restrict__ rf_out) { *rf_out = qs.rf[0]; }

}  // namespace geer

using namespace geer;

extern "C" geer_status geer_amc_device_noalloc(geer_graph *g, int32_t s, int32_t t, const void *d_xy,
                                               double eps, int32_t lf, int32_t tau, double delta,
                                               uint64_t seed, uint32_t q, uint32_t flags,
                                               void *stream, double *d_rf_out,
                                               geer_query_stats *d_stats)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (!d_xy || !d_rf_out) return fail(GEER_E_INVALID_ARG, "NULL array");
    if (s < 0 || s >= g->n || t < 0 || t >= g->n) return fail(GEER_E_INVALID_ARG, "node out of range");
    if (!(eps > 0.0) || std::isinf(eps)) return fail(GEER_E_INVALID_ARG, "eps must be > 0");
    if (lf < 0) return fail(GEER_E_INVALID_ARG, "lf must be >= 0");
    if (tau < 1 || tau > 30) return fail(GEER_E_INVALID_ARG, "tau must be in 1..30");
    if (!(delta > 0.0 && delta < 1.0)) return fail(GEER_E_INVALID_ARG, "delta must be in (0,1)");
    if (flags & ~(uint32_t)GEER_FLAG_FP64_VECTORS) return fail(GEER_E_INVALID_ARG, "unknown flags");
    GEER_HIP(hipSetDevice(g->device));
    unsigned char *base = nullptr;
    GEER_TRY(scratch_on_device(g->device, &base));
    hipStream_t st = stream ? (hipStream_t)stream : g->stream;
    const int vs = (flags & GEER_FLAG_FP64_VECTORS) ? 8 : 4;

    // the vectors must be finite and non-negative (checked on the device)
    uint32_t *d_bad = reinterpret_cast<uint32_t *>(base + kScrBad);
    hipLaunchKernelGGL(k_clear_flag, dim3(1), dim3(1), 0, st, d_bad);
    GEER_HIP(hipGetLastError());
    const int64_t count = 2 * (int64_t)g->n;
    const int cblocks = (int)std::min<int64_t>((count + 255) / 256, (int64_t)g->num_cus * 4);
    if (vs == 4)
        hipLaunchKernelGGL(k_check_vectors<float>, dim3(cblocks), dim3(256), 0, st, (const float *)d_xy,
                           count, d_bad);
    else
        hipLaunchKernelGGL(k_check_vectors<double>, dim3(cblocks), dim3(256), 0, st,
                           (const double *)d_xy, count, d_bad);
    GEER_HIP(hipGetLastError());
    uint32_t bad = 0;
    GEER_HIP(hipMemcpyAsync(&bad, d_bad, sizeof(bad), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    if (bad) return fail(GEER_E_INVALID_ARG, "vectors must be finite and non-negative");

    QueryCtx c;
    qstate_carve(reinterpret_cast<char *>(base + kScrQState), 1, &c.qs);
    c.nq = 1;
    c.lambda = 0.5;
    c.delta = delta;
    c.tau = tau;
    c.schedule = GEER_SCHEDULE_FIXED;
    c.seed = seed;
    c.qid_offset = (int64_t)q;  // the walk counter id is q + qid_offset with q = 0
    c.stream = st;
    double *cs_m1 = reinterpret_cast<double *>(base + kScrColstat);
    GEER_TRY(launch_column_top2(g, d_xy, 2, 2, vs, cs_m1, cs_m1 + kCols, st));
    GEER_TRY(launch_amc_setup(g, c.qs, s, t, lf, eps, tau, delta, 0, cs_m1, cs_m1 + kCols, st));
    AmcGroup grp;
    grp.q0 = 0;
    grp.nq = 1;
    grp.pool = d_xy;
    grp.value_size = vs;
    grp.vstride = 2;
    AmcScratch ext;
    ext.chunk_off = reinterpret_cast<int64_t *>(base + kScrChunkOff);
    ext.misc = reinterpret_cast<int64_t *>(base + kScrMisc);
    ext.zpart = reinterpret_cast<double2 *>(base + kScrZpart);
    ext.zpart_cap = kScrZpartCap;
    GEER_TRY(amc_phase(g, c, grp, st, 0, &ext));
    GEER_TRY(launch_finalize(g, c, reinterpret_cast<double *>(base + kScrR), d_stats, st));
    hipLaunchKernelGGL(k_amc_result, dim3(1), dim3(1), 0, st, c.qs, d_rf_out);
    GEER_HIP(hipGetLastError());
    GEER_HIP(hipStreamSynchronize(st));
    return GEER_OK;
}
