// Graph residency: validation of the canonical CSR, upload to HBM, inverse
// degrees, and the SpMM work decomposition (light rows / heavy-row segments).
#include <algorithm>
#include <atomic>
#include <cmath>
#include <cstring>
#include <numeric>
#include <thread>

#include "geer_internal.h"

namespace geer {

static thread_local std::string g_last_error;

void set_error(const std::string &msg) { g_last_error = msg; }

geer_status fail(geer_status st, const std::string &msg)
{
    g_last_error = msg;
    return st;
}

thread_local bool t_capturing = false;

std::vector<DevBuf *> workspace_bufs(geer_graph *g)
{
    Workspace &w = g->ws;
    return {&w.pool, &w.bits,   &w.part, &w.segbuf, &w.colstat, &w.qstate, &w.chunk_off,
            &w.zpart, &w.misc, &w.io,   &w.acc,    &w.meta,    &w.feat,   &w.hpart,
            &w.wfilter};
}

geer_status DevBuf::reserve(size_t want)
{
    if (want <= bytes) return GEER_OK;
    if (t_capturing) return fail(GEER_E_DEVICE, "buffer growth requested while capturing a launch graph");
    release();
    size_t cap = want + want / 8 + 256;
    hipError_t e = hipMalloc(&ptr, cap);
    if (e != hipSuccess) {
        ptr = nullptr;
        (void)hipGetLastError();
        return fail(GEER_E_OOM, "device allocation of " + std::to_string(cap) + " bytes failed");
    }
    bytes = cap;
    return GEER_OK;
}

void DevBuf::release()
{
    if (ptr && dependent && *dependent) {
        (void)hipGraphExecDestroy(*dependent);
        *dependent = nullptr;
    }
    if (ptr) (void)hipFree(ptr);
    ptr = nullptr;
    bytes = 0;
}

static hipEvent_t take_event(Profiler &p)
{
    if (!p.spare.empty()) {
        hipEvent_t e = p.spare.back();
        p.spare.pop_back();
        return e;
    }
    hipEvent_t e = nullptr;
    if (hipEventCreate(&e) != hipSuccess) return nullptr;
    return e;
}

int prof_begin(geer_graph *g, hipStream_t st)
{
    Profiler &p = g->prof;
    if (!p.on) return -1;
    ProfRec r{};
    r.a = take_event(p);
    r.b = take_event(p);
    if (!r.a || !r.b) return -1;
    if (hipEventRecord(r.a, st) != hipSuccess) return -1;
    p.recs.push_back(r);
    return (int)p.recs.size() - 1;
}

void prof_end(geer_graph *g, int token, int kind, double bytes, double units, hipStream_t st)
{
    Profiler &p = g->prof;
    if (!p.on || token < 0 || token >= (int)p.recs.size()) return;
    ProfRec &r = p.recs[token];
    r.kind = kind;
    r.bytes = bytes;
    r.units = units;
    (void)hipEventRecord(r.b, st);
}

void prof_add_units(geer_graph *g, int kind, double units, double bytes)
{
    if (g->prof.on) {
        g->prof.units[kind] += units;
        g->prof.bytes[kind] += bytes;
    }
}

static geer_status prof_flush(geer_graph *g)
{
    Profiler &p = g->prof;
    for (ProfRec &r : p.recs) GEER_HIP(hipEventSynchronize(r.b));
    std::vector<int64_t> cnt(2 * (size_t)p.n_counters);
    if (p.n_counters > 0)
        GEER_HIP(hipMemcpy(cnt.data(), p.d_counters, cnt.size() * sizeof(int64_t), hipMemcpyDeviceToHost));
    for (ProfRec &r : p.recs) {
        float ms = 0.f;
        GEER_HIP(hipEventElapsedTime(&ms, r.a, r.b));
        if (r.counter >= 0) {
            const double c0 = (double)cnt[2 * (size_t)r.counter], c1 = (double)cnt[2 * (size_t)r.counter + 1];
            r.bytes = r.per_unit * c0 + r.per_unit2 * c1;
            r.units = c0;
        }
        p.launches[r.kind] += 1;
        p.ms[r.kind] += ms;
        p.bytes[r.kind] += r.bytes;
        p.units[r.kind] += r.units;
        p.spare.push_back(r.a);
        p.spare.push_back(r.b);
    }
    p.recs.clear();
    p.n_counters = 0;
    return GEER_OK;
}

int64_t *prof_counter(geer_graph *g, int *index)
{
    Profiler &p = g->prof;
    *index = -1;
    if (!p.on) return nullptr;
    if (!p.d_counters) {
        if (hipMalloc(&p.d_counters, (size_t)kProfCounters * 2 * sizeof(int64_t)) != hipSuccess) {
            p.d_counters = nullptr;
            return nullptr;
        }
    }
    if (p.n_counters == kProfCounters && prof_flush(g) != GEER_OK) return nullptr;
    *index = p.n_counters++;
    return p.d_counters + 2 * (size_t)*index;
}

void prof_end_counted(geer_graph *g, int token, int kind, int counter, double per_unit,
                      double per_unit2, hipStream_t st)
{
    Profiler &p = g->prof;
    if (!p.on || token < 0 || token >= (int)p.recs.size()) return;
    ProfRec &r = p.recs[token];
    r.kind = kind;
    r.bytes = r.units = 0.0;
    r.counter = counter;
    r.per_unit = per_unit;
    r.per_unit2 = per_unit2;
    (void)hipEventRecord(r.b, st);
}

}  // namespace geer

using namespace geer;

// Host threads for the O(nnz) passes over the graph (canonical-form and
// connectivity checks, per-node tables): each reads random rows, so they are
// bound by memory latency and scale with threads.
static int host_threads()
{
    const unsigned hc = std::thread::hardware_concurrency();
    return (int)std::max(1u, std::min(16u, hc ? hc : 1u));
}

// Run f(lo, hi) over [0, n) split into `parts` contiguous ranges, one thread each.
template <class F> static void parallel_ranges(int64_t n, int parts, F f)
{
    parts = (int)std::max<int64_t>(1, std::min<int64_t>(parts, n));
    std::vector<std::thread> th;
    for (int i = 1; i < parts; ++i) th.emplace_back(f, n * i / parts, n * (i + 1) / parts);
    f(0, n / parts);
    for (auto &t : th) t.join();
}

static geer_status validate_csr(int32_t n, const int32_t *rp, const int32_t *ci)
{
    if (rp[0] != 0) return fail(GEER_E_GRAPH, "row_ptr[0] must be 0");
    for (int32_t v = 0; v < n; ++v) {
        if (rp[v + 1] < rp[v]) return fail(GEER_E_GRAPH, "row_ptr must be non-decreasing");
        if (rp[v + 1] == rp[v])
            return fail(GEER_E_GRAPH, "node " + std::to_string(v) + " has degree 0");
    }
    // canonical form per row (range, no self-loop, strictly ascending,
    // symmetric); the lowest failing row is reported
    const int T = host_threads();
    std::vector<int32_t> bad_row(T, n);
    std::vector<int> bad_kind(T, 0);
    std::vector<int32_t> bad_col(T, 0);
    std::atomic<int> part{0};
    parallel_ranges(n, T, [&](int64_t lo, int64_t hi) {
        const int me = part.fetch_add(1);
        for (int32_t v = (int32_t)lo; v < (int32_t)hi; ++v) {
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t u = ci[e];
                int kind = 0;
                if (u < 0 || u >= n) kind = 1;
                else if (u == v) kind = 2;
                else if (e > rp[v] && ci[e - 1] >= u) kind = 3;
                else if (!std::binary_search(ci + rp[u], ci + rp[u + 1], v)) kind = 4;
                if (kind) {
                    bad_row[me] = v;
                    bad_kind[me] = kind;
                    bad_col[me] = u;
                    return;
                }
            }
        }
    });
    int w = 0;
    for (int i = 1; i < T; ++i)
        if (bad_row[i] < bad_row[w]) w = i;
    if (bad_row[w] < n) {
        const int32_t v = bad_row[w], u = bad_col[w];
        switch (bad_kind[w]) {
        case 1: return fail(GEER_E_GRAPH, "col_idx out of range");
        case 2: return fail(GEER_E_GRAPH, "self-loop at node " + std::to_string(v));
        case 3:
            return fail(GEER_E_GRAPH, "row " + std::to_string(v) +
                                          " not strictly ascending (unsorted or duplicate)");
        default:
            return fail(GEER_E_GRAPH, "graph is not symmetric (" + std::to_string(v) + "," +
                                          std::to_string(u) + ")");
        }
    }
    // connectivity: level-synchronous breadth-first search from node 0, the
    // frontier split over threads, nodes claimed with an atomic flag
    std::vector<std::atomic<uint8_t>> seen(n);
    for (auto &f : seen) f.store(0, std::memory_order_relaxed);
    std::vector<int32_t> frontier{0};
    seen[0].store(1, std::memory_order_relaxed);
    int64_t reached = 1;
    while (!frontier.empty()) {
        std::vector<std::vector<int32_t>> next(T);
        std::atomic<int> slot{0};
        parallel_ranges((int64_t)frontier.size(), T, [&](int64_t lo, int64_t hi) {
            std::vector<int32_t> &out = next[slot.fetch_add(1)];
            for (int64_t h = lo; h < hi; ++h) {
                const int32_t u = frontier[h];
                for (int32_t e = rp[u]; e < rp[u + 1]; ++e) {
                    const int32_t x = ci[e];
                    if (!seen[x].load(std::memory_order_relaxed) &&
                        !seen[x].exchange(1, std::memory_order_relaxed))
                        out.push_back(x);
                }
            }
        });
        frontier.clear();
        for (auto &v : next) frontier.insert(frontier.end(), v.begin(), v.end());
        reached += (int64_t)frontier.size();
    }
    if (reached != n)
        return fail(GEER_E_NOT_CONNECTED, "graph is not connected (" + std::to_string(reached) +
                                              " of " + std::to_string(n) +
                                              " nodes reachable from 0)");
    return GEER_OK;
}

template <class T> static geer_status upload(T **dst, const T *src, size_t count)
{
    GEER_HIP(hipMalloc(dst, std::max<size_t>(count, 1) * sizeof(T)));
    if (count) GEER_HIP(hipMemcpy(*dst, src, count * sizeof(T), hipMemcpyHostToDevice));
    return GEER_OK;
}

__global__ void k_walk_records(int64_t nnz, const int32_t *__restrict__ row_ptr,
                               const int32_t *__restrict__ col_idx, int packed, uint32_t sb,
                               uint32_t sd, void *__restrict__ rec)
{
    for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < nnz;
         e += (int64_t)gridDim.x * blockDim.x) {
        const int32_t v = col_idx[e];
        const int32_t b = row_ptr[v], d = row_ptr[v + 1] - b;
        if (packed)
            static_cast<uint64_t *>(rec)[e] =
                (uint64_t)v | ((uint64_t)b << sb) | ((uint64_t)d << sd);
        else
            static_cast<int4 *>(rec)[e] = make_int4(v, b, d, 0);
    }
}

static int bit_width(uint64_t x)
{
    int k = 0;
    while (k < 64 && (1ull << k) <= x) ++k;
    return k;
}

static geer_status build_graph(geer_graph *g, const int32_t *rp, const int32_t *ci)
{
    const int32_t n = g->n;
    GEER_TRY(upload(&g->d_row_ptr, rp, (size_t)n + 1));
    GEER_TRY(upload(&g->d_col_idx, ci, (size_t)g->nnz));
    std::vector<float> invf(n);
    std::vector<double> invd(n);
    int32_t maxd = 0;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = rp[v + 1] - rp[v];
        maxd = std::max(maxd, d);
        invd[v] = 1.0 / (double)d;
        invf[v] = (float)invd[v];
    }
    g->max_deg = maxd;
    g->h_row_ptr.assign(rp, rp + n + 1);
    g->h_nbr_work.assign(n, 0);
    // hop-1 constants of each node u: the two smallest neighbour degrees
    // (1/d of them are the two largest entries of P e_u) and sum_{v in N(u)} d(v)
    std::vector<int32_t> mind(n, 0), mind2(n, 0);
    parallel_ranges(n, host_threads(), [&](int64_t lo, int64_t hi) {
        for (int32_t v = (int32_t)lo; v < (int32_t)hi; ++v) {
            int64_t w = 0;
            int32_t md = INT32_MAX, md2 = INT32_MAX;
            for (int32_t e = rp[v]; e < rp[v + 1]; ++e) {
                const int32_t du = rp[ci[e] + 1] - rp[ci[e]];
                w += du;
                if (du < md) {
                    md2 = md;
                    md = du;
                } else if (du < md2) {
                    md2 = du;
                }
            }
            g->h_nbr_work[v] = w;
            mind[v] = md;
            mind2[v] = md2 == INT32_MAX ? 0 : md2;
        }
    });
    GEER_TRY(upload(&g->d_nbr_work, g->h_nbr_work.data(), (size_t)n));
    GEER_TRY(upload(&g->d_min_nbr_deg, mind.data(), (size_t)n));
    GEER_TRY(upload(&g->d_nbr_deg2, mind2.data(), (size_t)n));
    // sparse-hop fixed point: a sum of at most max_deg terms, each <= 1, must fit 62 bits
    int bits = 0;
    while ((1ll << bits) <= (long long)maxd) ++bits;
    g->fx_shift = 62 - bits;
    GEER_TRY(upload(&g->d_inv_deg_f, invf.data(), invf.size()));
    GEER_TRY(upload(&g->d_inv_deg_d, invd.data(), invd.size()));
    {
        const int bv = std::max(1, bit_width((uint64_t)(n - 1)));
        const int bb = std::max(1, bit_width((uint64_t)std::max<int64_t>(g->nnz - 1, 0)));
        const int bd = bit_width((uint64_t)maxd);
        const bool packed = !g->wide_records && bv + bb + bd <= 64;
        g->walk_rec_bytes = packed ? 8 : 16;
        g->rec_sb = bv;
        g->rec_sd = bv + bb;
    }
    GEER_HIP(hipMalloc(&g->d_walk_rec, std::max<int64_t>(g->nnz, 1) * g->walk_rec_bytes));
    if (g->nnz) {
        const int64_t blocks = std::min<int64_t>((g->nnz + 255) / 256, 65536);
        hipLaunchKernelGGL(k_walk_records, dim3((unsigned)blocks), dim3(256), 0, g->stream,
                           g->nnz, g->d_row_ptr, g->d_col_idx, g->walk_rec_bytes == 8 ? 1 : 0,
                           (uint32_t)g->rec_sb, (uint32_t)g->rec_sd, g->d_walk_rec);
        GEER_HIP(hipGetLastError());
        GEER_HIP(hipStreamSynchronize(g->stream));
    }

    // light rows sorted by degree descending (long rows first for load balance),
    // heavy rows split into consecutive segments of at most kSegNnz entries
    std::vector<int32_t> light, heavy, seg_start, seg_b, seg_e;
    for (int32_t v = 0; v < n; ++v) {
        int32_t d = rp[v + 1] - rp[v];
        if (d > kSegNnz) {
            heavy.push_back(v);
            g->nnz_heavy += d;
        } else {
            light.push_back(v);
        }
    }
    std::stable_sort(light.begin(), light.end(), [&](int32_t a, int32_t b) {
        return rp[a + 1] - rp[a] > rp[b + 1] - rp[b];
    });
    seg_start.push_back(0);
    for (int32_t v : heavy) {
        for (int32_t b = rp[v]; b < rp[v + 1]; b += kSegNnz) {
            seg_b.push_back(b);
            seg_e.push_back(std::min(rp[v + 1], b + kSegNnz));
        }
        seg_start.push_back((int32_t)seg_b.size());
    }
    g->n_light = (int32_t)light.size();
    g->n_heavy = (int32_t)heavy.size();
    g->n_seg = (int32_t)seg_b.size();
    GEER_TRY(upload(&g->d_light_rows, light.data(), light.size()));
    GEER_TRY(upload(&g->d_heavy_rows, heavy.data(), heavy.size()));
    GEER_TRY(upload(&g->d_heavy_seg_start, seg_start.data(), seg_start.size()));
    GEER_TRY(upload(&g->d_seg_begin, seg_b.data(), seg_b.size()));
    GEER_TRY(upload(&g->d_seg_end, seg_e.data(), seg_e.size()));
    return GEER_OK;
}

extern "C" {

const char *geer_last_error(void) { return g_last_error.c_str(); }

const char *geer_version(void) { return "geer-mi355x 0.1 (gfx950)"; }

geer_status geer_graph_create(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              uint32_t flags, geer_graph **out)
{
    if (!out) return fail(GEER_E_INVALID_ARG, "out is NULL");
    *out = nullptr;
    if (n < 2) return fail(GEER_E_INVALID_ARG, "n must be >= 2");
    if (!row_ptr || !col_idx) return fail(GEER_E_INVALID_ARG, "row_ptr/col_idx is NULL");
    if (row_ptr[n] < 0) return fail(GEER_E_GRAPH, "row_ptr[n] is negative");
    if (flags & ~(uint32_t)(GEER_GRAPH_TRUSTED | GEER_GRAPH_WIDE_WALK_RECORDS))
        return fail(GEER_E_INVALID_ARG, "unknown graph flags");
    if (!(flags & GEER_GRAPH_TRUSTED)) GEER_TRY(validate_csr(n, row_ptr, col_idx));
    geer_graph *g = new geer_graph();
    g->n = n;
    g->wide_records = (flags & GEER_GRAPH_WIDE_WALK_RECORDS) != 0;
    g->nnz = row_ptr[n];
    if (hipGetDevice(&g->device) != hipSuccess) {
        delete g;
        return fail(GEER_E_DEVICE, "hipGetDevice failed (no GPU?)");
    }
    hipDeviceProp_t prop;
    if (hipGetDeviceProperties(&prop, g->device) != hipSuccess) {
        delete g;
        return fail(GEER_E_DEVICE, "hipGetDeviceProperties failed");
    }
    g->num_cus = prop.multiProcessorCount;
    for (DevBuf *b : workspace_bufs(g)) b->dependent = &g->gexec;
    if (hipStreamCreateWithFlags(&g->stream, hipStreamNonBlocking) != hipSuccess) {
        delete g;
        return fail(GEER_E_DEVICE, "hipStreamCreate failed");
    }
    bool ev_ok = hipStreamCreateWithFlags(&g->stream2, hipStreamNonBlocking) == hipSuccess;
    for (int i = 0; i < 2 && ev_ok; ++i)
        ev_ok = hipEventCreateWithFlags(&g->ev_smm[i], hipEventDisableTiming) == hipSuccess &&
                hipEventCreateWithFlags(&g->ev_clean[i], hipEventDisableTiming) == hipSuccess;
    if (ev_ok) ev_ok = hipEventCreateWithFlags(&g->pin_ev, hipEventDisableTiming) == hipSuccess;
    if (!ev_ok) {
        geer_graph_destroy(g);
        return fail(GEER_E_DEVICE, "stream or event creation failed");
    }
    geer_status st = build_graph(g, row_ptr, col_idx);
    if (st != GEER_OK) {
        std::string msg = geer_last_error();
        geer_graph_destroy(g);
        return fail(st, msg);
    }
    *out = g;
    return GEER_OK;
}

void geer_graph_destroy(geer_graph *g)
{
    if (!g) return;
    (void)hipSetDevice(g->device);
    if (g->stream) (void)hipStreamSynchronize(g->stream);
    void *ptrs[] = {g->d_row_ptr,    g->d_col_idx,    g->d_inv_deg_f,       g->d_inv_deg_d,
                    g->d_light_rows, g->d_heavy_rows, g->d_heavy_seg_start, g->d_seg_begin,
                    g->d_seg_end,    g->d_nbr_work,   g->d_min_nbr_deg,     g->d_walk_rec,
                    g->d_nbr_deg2};
    if (g->stream2) (void)hipStreamSynchronize(g->stream2);
    if (g->gexec) (void)hipGraphExecDestroy(g->gexec);
    g->gexec = nullptr;
    for (void *p : ptrs)
        if (p) (void)hipFree(p);
    for (DevBuf *b : workspace_bufs(g)) b->release();
    for (ProfRec &r : g->prof.recs) {
        (void)hipEventDestroy(r.a);
        (void)hipEventDestroy(r.b);
    }
    for (hipEvent_t e : g->prof.spare) (void)hipEventDestroy(e);
    if (g->prof.d_counters) (void)hipFree(g->prof.d_counters);
    for (int i = 0; i < 2; ++i) {
        if (g->ev_smm[i]) (void)hipEventDestroy(g->ev_smm[i]);
        if (g->ev_clean[i]) (void)hipEventDestroy(g->ev_clean[i]);
    }
    if (g->pin_ev) {
        (void)hipEventSynchronize(g->pin_ev);
        (void)hipEventDestroy(g->pin_ev);
    }
    if (g->h_pin) (void)hipHostFree(g->h_pin);
    if (g->stream2) (void)hipStreamDestroy(g->stream2);
    if (g->stream) (void)hipStreamDestroy(g->stream);
    delete g;
}

geer_status geer_profile_enable(geer_graph *g, int32_t on)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    GEER_TRY(prof_flush(g));
    Profiler &p = g->prof;
    p.on = on != 0;
    if (p.on) {
        for (int k = 0; k < PK_COUNT; ++k) {
            p.launches[k] = 0;
            p.ms[k] = p.bytes[k] = p.units[k] = 0.0;
        }
    }
    return GEER_OK;
}

geer_status geer_profile_read(geer_graph *g, geer_kernel_profile *out, int32_t cap, int32_t *count)
{
    if (!g || (!out && cap > 0)) return fail(GEER_E_INVALID_ARG, "NULL argument");
    GEER_TRY(prof_flush(g));
    static const char *names[PK_COUNT] = {"hop_light", "hop_segments", "hop_heavy_fin", "hop1",
                                          "colstat", "epilogue", "walk", "amc_plan", "amc_stop",
                                          "features", "mlp", "hop2_global", "hop2_lds", "dense_hop",
                                          "graph"};
    int32_t k = 0;
    for (int i = 0; i < PK_COUNT && k < cap; ++i) {
        geer_kernel_profile &r = out[k++];
        std::memset(&r, 0, sizeof(r));
        std::strncpy(r.name, names[i], sizeof(r.name) - 1);
        r.launches = g->prof.launches[i];
        r.total_ms = g->prof.ms[i];
        r.alg_bytes = g->prof.bytes[i];
        r.work_units = g->prof.units[i];
    }
    if (count) *count = k;
    return GEER_OK;
}

geer_status geer_graph_set_lambda(geer_graph *g, double lambda)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (!(lambda >= 0.0) || std::isnan(lambda))
        return fail(GEER_E_INVALID_ARG, "lambda must be a number >= 0");
    if (lambda >= 1.0) return fail(GEER_E_BIPARTITE, "lambda >= 1: graph is bipartite");
    g->lambda = lambda;
    g->has_lambda = true;
    return GEER_OK;
}

geer_status geer_graph_get_lambda(const geer_graph *g, double *lambda_out)
{
    if (!g || !lambda_out) return fail(GEER_E_INVALID_ARG, "NULL argument");
    if (!g->has_lambda) return fail(GEER_E_NO_LAMBDA, "lambda has not been set");
    *lambda_out = g->lambda;
    return GEER_OK;
}

geer_status geer_graph_info(const geer_graph *g, int32_t *n, int64_t *nnz, int32_t *max_degree)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (n) *n = g->n;
    if (nnz) *nnz = g->nnz;
    if (max_degree) *max_degree = g->max_deg;
    return GEER_OK;
}

}  // extern "C"
