// Query driver: batching of pairs into 64-pair SMM batches, groups of batches
// resident in HBM before each AMC phase, and the C entry points.
#include <algorithm>
#include <cmath>
#include <cstring>

#include "geer_internal.h"

namespace geer {

size_t qstate_bytes(int64_t cap)
{
    return (size_t)cap * (14 * sizeof(int32_t) + 14 * sizeof(int64_t)) + 64;
}

void qstate_carve(char *p, int64_t cap, QState *qs)
{
    auto take = [&](auto *&dst, size_t elem) {
        dst = reinterpret_cast<std::remove_reference_t<decltype(dst)>>(p);
        p += (size_t)cap * elem;
    };
    // 8-byte fields first keeps every array aligned
    take(qs->eta1, 8);
    take(qs->walk_pairs, 8);
    take(qs->supp_sum, 8);
    take(qs->vec_off, 8);
    take(qs->eps, 8);
    take(qs->rb, 8);
    take(qs->psi, 8);
    take(qs->eta_star, 8);
    take(qs->zsum, 8);
    take(qs->z2sum, 8);
    take(qs->var, 8);
    take(qs->f, 8);
    take(qs->rf, 8);
    take(qs->r, 8);
    take(qs->s, 4);
    take(qs->t, 4);
    take(qs->ell, 4);
    take(qs->lb, 4);
    take(qs->lb_target, 4);
    take(qs->lf, 4);
    take(qs->batches, 4);
    take(qs->stop, 4);
    take(qs->active_smm, 4);
    take(qs->active_amc, 4);
    take(qs->fallback, 4);
    take(qs->tau_q, 4);
    take(qs->ord, 4);
    take(qs->h1w, 4);
}

geer_status ensure_qstate(geer_graph *g, int64_t nq, QState *qs)
{
    Workspace &ws = g->ws;
    const int64_t cap = std::max<int64_t>(nq, 1);
    GEER_TRY(ws.qstate.reserve(qstate_bytes(cap)));
    GEER_TRY(ws.misc.reserve((kMiscWords + 1024) * sizeof(int64_t)));
    GEER_TRY(ws.colstat.reserve(kCols * (2 * sizeof(double) + sizeof(int64_t))));
    qstate_carve(ws.qstate.as<char>(), cap, qs);
    ws.nq_cap = cap;
    return GEER_OK;
}

// Slot buffers and hop-2 accumulators are all zero between calls.  A call
// that fails after filling them leaves `in_use` set; the next call then has
// them cleared again (by ensure_slots / ensure_hop2_acc) before any use.
static void begin_slot_use(geer_graph *g)
{
    if (g->ws.in_use) {
        g->ws.slots = 0;
        g->ws.acc_slots = 0;
    }
    g->ws.in_use = true;
}

geer_status ensure_slots(geer_graph *g, int slots, int value_size)
{
    Workspace &ws = g->ws;
    const size_t vals = (size_t)slots * 3 * (size_t)g->n * kCols;
    const size_t words = (size_t)slots * 3 * (size_t)g->n * kBitWords;
    const size_t vbytes = vals * (size_t)value_size, bbytes = words * sizeof(uint32_t);
    bool grow = vbytes > ws.pool.bytes || bbytes > ws.bits.bytes;
    if (grow || ws.value_size != value_size || ws.slots < slots) {
        GEER_TRY(ws.pool.reserve(vbytes));
        GEER_TRY(ws.bits.reserve(bbytes));
        // H1 buffers must start (and are kept) all zero; clear everything once
        GEER_HIP(hipMemset(ws.pool.ptr, 0, ws.pool.bytes));
        GEER_HIP(hipMemset(ws.bits.ptr, 0, ws.bits.bytes));
        ws.slots = slots;
        ws.value_size = value_size;
        ws.a_dirty.assign(slots, 0);
    }
    if ((int)ws.a_dirty.size() < slots) ws.a_dirty.resize(slots, 0);
    GEER_TRY(ws.colstat.reserve((size_t)std::max(slots, 1) * kCols * (2 * sizeof(double) + sizeof(int64_t))));
    GEER_TRY(ws.hpart.reserve((size_t)std::max(slots, 1) * 3 * kPushSplitMax * kCols * sizeof(double)));
    return GEER_OK;
}

// Active-pair mask of every batch of a group (block k -> mask word k).
__global__ void k_batch_mask(QState qs, SlotArgs sa)
{
    const int k = blockIdx.x, j = threadIdx.x;
    const bool a = j < slot_nb(sa, k) && qs.active_smm[qs.ord[slot_q0(sa, k) + j]];
    const unsigned long long m = __ballot(a);
    if (j == 0) sa.meta[k] = m;
}

// Small host-computed mask words go to the device as kernel arguments: no
// pageable-memory copy whose source must outlive the call, and nothing that
// stream capture could not record.
struct Words64 {
    uint64_t w[64];
};

__global__ void k_set_words(uint64_t *__restrict__ dst, int n, Words64 v)
{
    if ((int)threadIdx.x < n) dst[threadIdx.x] = v.w[threadIdx.x];
}

static geer_status set_words(uint64_t *dst, const uint64_t *src, size_t n, hipStream_t st)
{
    for (size_t i = 0; i < n; i += 64) {
        Words64 v;
        const int m = (int)std::min<size_t>(64, n - i);
        std::memcpy(v.w, src + i, m * sizeof(uint64_t));
        hipLaunchKernelGGL(k_set_words, dim3(1), dim3(64), 0, st, dst + i, m, v);
        GEER_HIP(hipGetLastError());
    }
    return GEER_OK;
}

struct SlotView {
    char *pool;      // slot 0 of this slot set
    uint32_t *bits;
    size_t n;
    int vs;
    int k0 = 0;      // index of slot 0 among all slots (per-slot flags and statistics)
    void *buf(int slot, int which) const
    {
        return pool + ((size_t)slot * 3 + which) * n * kCols * vs;
    }
    int64_t elem_off(int slot, int which) const { return ((int64_t)slot * 3 + which) * (int64_t)n * kCols; }
    uint32_t *bw(int slot, int which) const { return bits + ((size_t)slot * 3 + which) * n * kBitWords; }
};

// What a batch left in its slot (needed to restore the all-zero state of the
// sparse buffers after the group's AMC phase).
struct BatchRec {
    bool hop1 = false;          // H1 holds scattered entries of every pair
    bool hop1_sel = false;      // H1 may hold entries of the pairs flagged in h1w
    uint64_t hop2_sparse = 0;   // pairs whose hop-2 vectors were pushed into A
};

// Per-slot device words (G = slots of the layout): [0,G) active masks,
// [G,2G) hop-2 masks, [2G,6G) hop-2 paths (LDS columns: 2 words, global
// columns: 2 words), [6G, 6G + G*L) static level masks.
struct SlotMeta {
    uint64_t *base;
    int G;
    uint64_t *active(int k) const { return base + k; }
    uint64_t *h2(int k) const { return base + G + k; }
    uint64_t *level(int k, int h, int L) const { return base + 6 * G + (size_t)k * L + h; }
};

// Host view of one group: which batch sits in which slot and its queries.
struct GroupPlan {
    int64_t p0 = 0, nbat = 0;  // first position and batch count
    int64_t pend = 0;          // end of the phase (positions)
    int B = 64;
};

static SlotArgs slot_args(geer_graph *g, const SlotView &sv, const SlotMeta &sm, const GroupPlan &gp)
{
    SlotArgs a;
    a.p0 = gp.p0;
    a.pend = gp.pend;
    a.B = gp.B;
    a.G = sm.G;
    a.pool = sv.pool;
    a.bits = sv.bits;
    a.buf_elems = (int64_t)sv.n * kCols;
    a.buf_words = (int64_t)sv.n * kBitWords;
    a.cs = g->ws.colstat.as<double>() + (size_t)sv.k0 * 3 * kCols;
    a.hpart = g->ws.hpart.as<double>() + (size_t)sv.k0 * 3 * kPushSplitMax * kCols;
    a.meta = sm.base;
    return a;
}

// Column tile of one dense hop.  An explicit request wins; with measured
// tile times the cheapest is taken for this hop's active pairs (only tiles
// holding an active pair are launched); otherwise the default.
static int pick_tile(const geer_graph *g, int requested, uint64_t hmask, int vs)
{
    if (requested < 0) return -requested;  // forced by the caller
    if (vs != 4 || g->tile_ns[0] <= 0.0) return requested;
    const int kts[3] = {32, 64, 128};
    double best = 1e300;
    int pick = requested;
    for (int i = 0; i < 3; ++i) {
        const int kt = kts[i];
        int tiles = 0;
        for (int c0 = 0; c0 < kCols; c0 += kt) {
            const uint64_t tp = kt == 128 ? ~0ull : (((1ull << (kt / 2)) - 1ull) << (c0 / 2));
            tiles += (hmask & tp) ? 1 : 0;
        }
        const double cost = tiles * g->tile_ns[i];
        if (cost < best) {
            best = cost;
            pick = kt;
        }
    }
    return pick;
}

// One hop level (hop >= 2) of the batches [0, nbat) of a group.  hm[k]: pairs
// of batch k active at this hop; dmask[k]: the same mask on the device.
// Hop 2 of a batch is sparse (exact push from the hop-1 frontier) when its
// work, the neighbour-degree sums of its start nodes, is at most two passes
// over the CSR; columns whose work fits an LDS hash table take the LDS path,
// the others the global fixed-point path.  One launch covers every batch for
// the LDS path, the statistics and the epilogue; dense hops run per batch.
static geer_status run_level(geer_graph *g, const QueryCtx &c, const SlotView &sv,
                             const SlotMeta &sm, const SlotArgs &sa, int nbat, int hop,
                             const std::vector<uint64_t> &hm,
                             const std::vector<const uint64_t *> &dmask, const int32_t *h_s,
                             const int32_t *h_t, const int32_t *h_ord, int col_tile,
                             std::vector<BatchRec> &recs)
{
    Workspace &ws = g->ws;
    const int L = sm.G;
    const int wout = hop % 2 == 0 ? 1 : 2;  // output buffer: A on even hops, B on odd
    std::vector<char> sparse(nbat, 0);
    if (hop == 2 && sv.vs == 4) {
        std::vector<uint64_t> words(5 * (size_t)L, 0);  // h2 masks, then paths
        bool any = false, any_lds = false;
        std::vector<char> glob(nbat, 0);
        int nglob = 0;  // global-path columns of the level
        for (int k = 0; k < nbat; ++k) {
            if (!hm[k]) continue;
            uint64_t m_lds[2] = {0, 0}, m_glob[2] = {0, 0};
            double work = 0.0, work_lds = 0.0;
            const int64_t q0 = slot_q0(sa, k);
            for (int j = 0; j < slot_nb(sa, k); ++j) {
                if (!((hm[k] >> j) & 1ull)) continue;
                const int32_t q = h_ord[q0 + j];
                for (int side = 0; side < 2; ++side) {
                    const int c2 = 2 * j + side;
                    const int64_t wk = g->h_nbr_work[side ? h_t[q] : h_s[q]];
                    work += (double)wk;
                    if (wk <= kHashLoadMax) {
                        m_lds[c2 >> 6] |= 1ull << (c2 & 63);
                        work_lds += (double)wk;
                    } else {
                        m_glob[c2 >> 6] |= 1ull << (c2 & 63);
                    }
                }
            }
            if (work > 2.0 * (double)g->nnz) continue;
            sparse[k] = 1;
            any = true;
            any_lds |= (m_lds[0] | m_lds[1]) != 0;
            glob[k] = (m_glob[0] | m_glob[1]) != 0;
            nglob += __builtin_popcountll(m_glob[0]) + __builtin_popcountll(m_glob[1]);
            words[k] = hm[k];
            uint64_t *pw = &words[L + 4 * (size_t)k];
            pw[0] = m_lds[0];
            pw[1] = m_lds[1];
            pw[2] = m_glob[0];
            pw[3] = m_glob[1];
            // algorithmic bytes of the push: per unit (one CSR entry of a
            // neighbour's row) its 4-byte index and an 8-byte accumulator update
            prof_add_units(g, PK_HOP2_LDS, work_lds, kHop2UnitBytes * work_lds);
            prof_add_units(g, PK_HOP2_SPARSE, work - work_lds, kHop2UnitBytes * (work - work_lds));
        }
        if (any) {
            for (int k = 0; k < nbat; ++k)
                if (sparse[k] && ws.a_dirty[sv.k0 + k]) {
                    GEER_TRY(launch_zero(g, sv.buf(k, 1), (size_t)g->n * kCols * sv.vs, c.stream));
                    GEER_TRY(launch_zero(g, sv.bw(k, 1), (size_t)g->n * kBitWords * 4, c.stream));
                    ws.a_dirty[sv.k0 + k] = 0;
                }
            GEER_TRY(set_words(sm.h2(0), words.data(), words.size(), c.stream));
            GEER_TRY(launch_zero(g, sa.hpart, (size_t)nbat * 3 * kPushSplitMax * kCols * sizeof(double),
                                 c.stream));
            if (any_lds) GEER_TRY(launch_hop2_lds_group(g, c, sa, nbat, sv.vs, c.stream));
            int k0 = 0, k1 = -1;  // slots with global-path columns lie in [k0, k1]
            for (int k = nbat - 1; k >= 0; --k)
                if (glob[k]) k0 = k;
            for (int k = 0; k < nbat; ++k)
                if (glob[k]) k1 = k;
            const int split = hop2_split(nglob);
            if (k1 >= k0) {
                geer_status err;
                const int A = ensure_hop2_acc(g, k1 - k0 + 1, c.stream, &err);
                GEER_TRY(err);
                for (int a0 = k0; a0 <= k1; a0 += A) {
                    const int na = std::min(A, k1 + 1 - a0);
                    GEER_TRY(launch_hop2_sparse(g, c, sa, a0, na, sv.vs, 0, split, c.stream));
                    GEER_TRY(launch_hop2_sparse(g, c, sa, a0, na, sv.vs, 1, split, c.stream));
                }
            }
            GEER_TRY(launch_colstat_group(g, sa, nbat, split, c.stream));
            for (int k = 0; k < nbat; ++k)
                if (sparse[k]) recs[k].hop2_sparse = hm[k];
        }
    }
    for (int k = 0; k < nbat; ++k) {
        if (!hm[k] || sparse[k]) continue;
        const int win = hop == 2 ? 0 : (hop % 2 == 0 ? 2 : 1);
        // a dense hop 2 gathers from H1: scatter it for the pairs going on
        if (hop == 2 && c.hop1_implicit)
            GEER_TRY(launch_hop1_select(g, c, sa, k, 1, kHop1Continuing, c.stream));
        HopArgs a;
        a.in = sv.buf(k, win);
        a.out = sv.buf(k, wout);
        a.in_bits = sv.bw(k, win);
        a.out_bits = sv.bw(k, wout);
        a.mask = dmask[k];
        a.host_mask = hm[k];
        a.cs = slot_cs(sa, k);
        a.col0 = 0;
        a.col_tile = pick_tile(g, col_tile, hm[k], sv.vs);
        GEER_TRY(launch_hop_dense(g, a, sv.vs, c.stream));
        if (wout == 1) ws.a_dirty[sv.k0 + k] = 1;
    }
    return launch_epilogue_group(g, c, sa, nbat, hop, wout, sv.vs, c.stream);
}

// Restore H1 and the sparse part of A of the group's batches to zero.
static geer_status cleanup_group(geer_graph *g, const QueryCtx &c, const SlotView &sv,
                                 const SlotMeta &sm, const SlotArgs &sa, int nbat,
                                 const std::vector<BatchRec> &recs)
{
    bool h1 = false, h1s = false, h2 = false;
    int ncols = 0;
    std::vector<uint64_t> words(nbat, 0);
    for (int k = 0; k < nbat; ++k) {
        h1 |= recs[k].hop1;
        h1s |= recs[k].hop1_sel;
        // a dense hop that wrote A later makes it dirty: it is zeroed in full
        // before its next sparse use instead
        if (recs[k].hop2_sparse && !g->ws.a_dirty[sv.k0 + k]) {
            words[k] = recs[k].hop2_sparse;
            ncols += 2 * __builtin_popcountll(words[k]);
            h2 = true;
        }
    }
    if (h1) GEER_TRY(launch_hop1_group(g, c, sa, nbat, true, c.stream));
    if (h1s) GEER_TRY(launch_hop1_select(g, c, sa, 0, nbat, kHop1Clear, c.stream));
    if (h2) {
        GEER_TRY(set_words(sm.h2(0), words.data(), words.size(), c.stream));
        GEER_TRY(launch_hop2_sparse(g, c, sa, 0, nbat, sv.vs, 2, hop2_split(ncols), c.stream));
    }
    return GEER_OK;
}

// SMM of a group of batches.  Greedy: level-synchronous, one host read of the
// batch masks per hop level.  Static (fixed / learned depths known on the
// host): the whole launch sequence is fixed in advance, no host reads.
static geer_status smm_group(geer_graph *g, const QueryCtx &c, const SlotView &sv,
                             const SlotMeta &sm, const GroupPlan &gp, bool is_static,
                             const int32_t *h_target, const int32_t *h_s, const int32_t *h_t,
                             const int32_t *h_ord, int col_tile, int max_hops,
                             std::vector<BatchRec> &recs)
{
    const int nbat = (int)gp.nbat;
    for (int k = 0; k < nbat; ++k) recs[k] = BatchRec();
    const SlotArgs sa = slot_args(g, sv, sm, gp);
    std::vector<uint64_t> hm(nbat, 0);
    std::vector<const uint64_t *> dmask(nbat, nullptr);
    if (is_static) {
        // level masks from the known depths
        int L = 1;
        for (int k = 0; k < nbat; ++k)
            for (int j = 0; j < slot_nb(sa, k); ++j) L = std::max(L, h_target[h_ord[slot_q0(sa, k) + j]] + 1);
        if ((6 * (size_t)sm.G + (size_t)sm.G * L) * 8 > g->ws.meta.bytes)
            return fail(GEER_E_DEVICE, "mask words exceed their reservation");
        std::vector<uint64_t> lv((size_t)nbat * L, 0);
        for (int k = 0; k < nbat; ++k)
            for (int j = 0; j < slot_nb(sa, k); ++j) {
                const int t = h_target[h_ord[slot_q0(sa, k) + j]];
                for (int h = 1; h <= t && h < L; ++h) lv[(size_t)k * L + h] |= 1ull << j;
            }
        if (L < 2) return GEER_OK;
        GEER_TRY(set_words(sm.level(0, 0, L), lv.data(), lv.size(), c.stream));
        if (c.hop1_implicit) {
            GEER_TRY(launch_epilogue_group(g, c, sa, nbat, 1, 0, sv.vs, c.stream));
            GEER_TRY(launch_hop1_select(g, c, sa, 0, nbat, kHop1Stopped, c.stream));
            for (int k = 0; k < nbat; ++k) recs[k].hop1_sel = lv[(size_t)k * L + 1] != 0;
        } else {
            GEER_TRY(launch_hop1_group(g, c, sa, nbat, false, c.stream));
            for (int k = 0; k < nbat; ++k) recs[k].hop1 = lv[(size_t)k * L + 1] != 0;
            GEER_TRY(launch_epilogue_group(g, c, sa, nbat, 1, 0, sv.vs, c.stream));
        }
        for (int h = 2; h < L; ++h) {
            bool any = false;
            for (int k = 0; k < nbat; ++k) {
                hm[k] = lv[(size_t)k * L + h];
                dmask[k] = sm.level(k, h, L);
                any |= hm[k] != 0;
            }
            if (any)
                GEER_TRY(run_level(g, c, sv, sm, sa, nbat, h, hm, dmask, h_s, h_t, h_ord, col_tile, recs));
        }
        return GEER_OK;
    }
    // greedy: level 1 for every batch, then one read of all masks per level
    hipLaunchKernelGGL(k_batch_mask, dim3(nbat), dim3(64), 0, c.stream, c.qs, sa);
    GEER_HIP(hipGetLastError());
    if (c.hop1_implicit) {
        GEER_TRY(launch_epilogue_group(g, c, sa, nbat, 1, 0, sv.vs, c.stream));
        GEER_TRY(launch_hop1_select(g, c, sa, 0, nbat, kHop1Stopped, c.stream));
    } else {
        GEER_TRY(launch_hop1_group(g, c, sa, nbat, false, c.stream));
        GEER_TRY(launch_epilogue_group(g, c, sa, nbat, 1, 0, sv.vs, c.stream));
    }
    for (int k = 0; k < nbat; ++k) {
        recs[k].hop1 = !c.hop1_implicit;
        recs[k].hop1_sel = c.hop1_implicit;
        dmask[k] = sm.active(k);
    }
    for (int hop = 2;; ++hop) {
        GEER_HIP(hipMemcpyAsync(hm.data(), sm.active(0), nbat * sizeof(uint64_t), hipMemcpyDeviceToHost,
                                c.stream));
        GEER_HIP(hipStreamSynchronize(c.stream));
        bool any = false;
        for (int k = 0; k < nbat; ++k) any |= hm[k] != 0;
        if (!any) break;
        if (hop > max_hops)
            return fail(GEER_E_DEVICE, "SMM batch still active after the largest possible l");
        GEER_TRY(run_level(g, c, sv, sm, sa, nbat, hop, hm, dmask, h_s, h_t, h_ord, col_tile, recs));
    }
    return GEER_OK;
}

static int default_col_tile(const geer_graph *g, int vs)
{
    if (g->tuned_col_tile && vs == 4) return g->tuned_col_tile;
    // keep one column tile of the vectors within the 256 MB last-level cache
    const double tile_bytes_128 = (double)g->n * kCols * vs;
    if (tile_bytes_128 <= 96e6) return 128;
    if (tile_bytes_128 / 2 <= 96e6) return 64;
    return 32;
}

static int default_group_batches(const geer_graph *g, int vs, int64_t nbatches, int sets)
{
    // up to 32 batches (2,048 pairs) share one AMC phase; the slot buffers of
    // all slot sets within ~96 GB (one set) or ~128 GB (two sets) of the
    // 288 GB of HBM (the hop-2 accumulators take at most a quarter of the rest)
    const double slot_bytes = 3.0 * g->n * kCols * vs;
    const double budget = sets == 2 ? 128e9 : 96e9;
    int grp = (int)std::max(1.0, std::min(32.0, budget / (sets * slot_bytes)));
    return (int)std::min<int64_t>(grp, std::max<int64_t>(nbatches, 1));
}

static geer_status check_params(const geer_params &p)
{
    if (!(p.delta > 0.0 && p.delta < 1.0)) return fail(GEER_E_INVALID_ARG, "delta must be in (0,1)");
    if (p.tau < 1 || p.tau > 30) return fail(GEER_E_INVALID_ARG, "tau must be in 1..30");
    if (p.schedule != GEER_SCHEDULE_GREEDY && p.schedule != GEER_SCHEDULE_FIXED &&
        p.schedule != GEER_SCHEDULE_LEARNED)
        return fail(GEER_E_INVALID_ARG, "unknown schedule");
    if (p.batch_queries < 0 || p.batch_queries > kMaxPairs)
        return fail(GEER_E_INVALID_ARG, "batch_queries must be in 0..64");
    if (p.col_tile != 0 && p.col_tile != 32 && p.col_tile != 64 && p.col_tile != 128)
        return fail(GEER_E_INVALID_ARG, "col_tile must be 0, 32, 64 or 128");
    if (p.group_batches < 0) return fail(GEER_E_INVALID_ARG, "group_batches must be >= 0");
    if (p.walk_ilp != 0 && p.walk_ilp != 1) return fail(GEER_E_INVALID_ARG, "walk_ilp must be 0 or 1");
    if (p.flags & ~(uint32_t)(GEER_FLAG_FP64_VECTORS | GEER_FLAG_GRAPH_LAUNCH | GEER_FLAG_PENG_ELL))
        return fail(GEER_E_INVALID_ARG, "unknown flags");
    if (p.schedule == GEER_SCHEDULE_LEARNED && !p.model)
        return fail(GEER_E_MODEL, "LEARNED schedule needs a model");
    return GEER_OK;
}

// Everything a captured call's launches were derived from, as bytes: a later
// call deriving the same bytes replays the captured graph.
struct GraphSig {
    std::vector<unsigned char> b;
    template <class T> void add(const T &v)
    {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(&v);
        b.insert(b.end(), p, p + sizeof(T));
    }
    template <class T> void add_n(const T *v, size_t n)
    {
        const unsigned char *p = reinterpret_cast<const unsigned char *>(v);
        b.insert(b.end(), p, p + n * sizeof(T));
    }
};

// The whole query pipeline on device-resident inputs (already in qstate).
// h_s / h_t: host copies of the pairs (used for planning only).
// Pinned host staging of at least `bytes` (grown as needed).  Waits for the
// last copy that read it, so the host may overwrite it.
static geer_status pinned_staging(geer_graph *g, size_t bytes, char **out)
{
    GEER_HIP(hipEventSynchronize(g->pin_ev));
    if (bytes > g->h_pin_bytes) {
        if (g->h_pin) GEER_HIP(hipHostFree(g->h_pin));
        g->h_pin = nullptr;
        g->h_pin_bytes = 0;
        const size_t cap = bytes + bytes / 4 + 4096;
        GEER_HIP(hipHostMalloc((void **)&g->h_pin, cap, hipHostMallocDefault));
        g->h_pin_bytes = cap;
    }
    *out = g->h_pin;
    return GEER_OK;
}

static geer_status run_queries(geer_graph *g, QueryCtx &c, const geer_params &p,
                               const int32_t *d_fixed, double min_eps, const int32_t *h_s,
                               const int32_t *h_t)
{
    begin_slot_use(g);
    c.hop1_implicit = true;
    // no pair can need more products than l of Eq. (ell) at d(s) = d(t) = 1
    const int max_hops = ell_of(1.0, 1.0, min_eps, c.lambda);
    const int vs = (p.flags & GEER_FLAG_FP64_VECTORS) ? 8 : 4;
    const int B = p.batch_queries ? p.batch_queries : kMaxPairs;
    const int64_t nbatches = (c.nq + B - 1) / B;
    // one slot set when every batch fits one group, else two: group i + 1's
    // SMM fills one set while group i's AMC phase reads the other
    int G = std::min(1024, p.group_batches ? p.group_batches : default_group_batches(g, vs, nbatches, 1));
    const int sets = nbatches > G ? 2 : 1;
    if (sets == 2 && !p.group_batches) G = default_group_batches(g, vs, nbatches, 2);
    const int col_tile = p.col_tile ? -p.col_tile : default_col_tile(g, vs);
    GEER_TRY(ensure_slots(g, sets * G, vs));
    const size_t meta_words = 6 * (size_t)G + (size_t)G * (max_hops + 2);
    GEER_TRY(g->ws.meta.reserve((sets * meta_words) * 8 + 64));
    GEER_TRY(launch_init_queries(g, c, d_fixed, -1, c.stream));
    const bool learned = p.schedule == GEER_SCHEDULE_LEARNED;
    if (learned) c.tau = std::max(c.tau, kLearnedTauMax);
    // GEER_FLAG_GRAPH_LAUNCH: the groups with known depths run as one
    // captured graph (a greedy schedule has none)
    const bool graph_mode = (p.flags & GEER_FLAG_GRAPH_LAUNCH) && p.schedule != GEER_SCHEDULE_GREEDY;
    std::vector<int32_t> ord(c.nq), target(c.nq, 0), taus(graph_mode ? c.nq : 0);
    for (int64_t i = 0; i < c.nq; ++i) ord[i] = (int32_t)i;
    int64_t n_static = 0;  // positions [0, n_static) run a static plan, the rest greedy
    if (p.schedule != GEER_SCHEDULE_GREEDY) {
        if (learned) {
            GEER_TRY(g->ws.feat.reserve((size_t)c.nq * GEER_MLP_FEATURES * sizeof(float)));
            GEER_TRY(launch_learned(g, c, p.model, g->ws.feat.as<float>(), c.tau, c.stream));
        }
        // depths are known: bucket pairs of equal SMM depth into the same
        // batches so that dense hops run on full batches, shallowest first
        // (the first group needs hop 1 only, so walks start at once)
        // one copy of the per-pair int32 arrays from ell to tau_q (they are
        // consecutive in the query state) into pinned host memory
        const int32_t *base = c.qs.ell;
        const size_t span = (size_t)(c.qs.tau_q - base) + (size_t)c.nq;
        char *pin = nullptr;
        GEER_TRY(pinned_staging(g, span * sizeof(int32_t), &pin));
        GEER_HIP(hipMemcpyAsync(pin, base, span * sizeof(int32_t), hipMemcpyDeviceToHost, c.stream));
        GEER_HIP(hipStreamSynchronize(c.stream));
        const int32_t *h = reinterpret_cast<const int32_t *>(pin);
        auto host = [&](const int32_t *dev) { return h + (dev - base); };
        const int32_t *tgt = host(c.qs.lb_target), *ellh = host(c.qs.ell), *act = host(c.qs.active_smm);
        const int32_t *fbh = host(c.qs.fallback), *tq = host(c.qs.tau_q);
        std::vector<int32_t> fb(fbh, fbh + c.nq);
        for (int64_t i = 0; i < c.nq; ++i) target[i] = act[i] ? std::min(tgt[i], ellh[i]) : 0;
        if (graph_mode) std::copy(tq, tq + c.nq, taus.begin());
        std::stable_sort(ord.begin(), ord.end(), [&](int32_t a, int32_t b) {
            if (fb[a] != fb[b]) return fb[a] < fb[b];  // fallback pairs last
            return target[a] < target[b];
        });
        n_static = 0;
        while (n_static < c.nq && !fb[ord[n_static]]) ++n_static;
    }
    if (p.schedule != GEER_SCHEDULE_GREEDY) {
        // the staging buffer was read above (after its last upload completed)
        char *pin = nullptr;
        GEER_TRY(pinned_staging(g, (size_t)c.nq * sizeof(int32_t), &pin));
        std::memcpy(pin, ord.data(), (size_t)c.nq * sizeof(int32_t));
        GEER_HIP(hipMemcpyAsync(c.qs.ord, pin, c.nq * sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
        GEER_HIP(hipEventRecord(g->pin_ev, c.stream));
    } else {
        GEER_HIP(hipMemcpyAsync(c.qs.ord, ord.data(), c.nq * sizeof(int32_t), hipMemcpyHostToDevice, c.stream));
    }
    // groups in order: the static phase (known depths), then the greedy one
    struct Job {
        GroupPlan gp;
        bool is_static;
        int set;
    };
    std::vector<Job> jobs;
    for (int phase = 0; phase < 2; ++phase) {
        const bool is_static = phase == 0;
        const int64_t pb = is_static ? 0 : n_static, pe = is_static ? n_static : c.nq;
        const int64_t nbat_phase = (pe - pb + B - 1) / B;
        for (int64_t b0 = 0; b0 < nbat_phase; b0 += G) {
            Job jb;
            jb.gp.p0 = pb + b0 * B;
            jb.gp.nbat = std::min<int64_t>(nbat_phase, b0 + G) - b0;
            jb.gp.pend = pe;
            jb.gp.B = B;
            jb.is_static = is_static;
            jobs.push_back(jb);
        }
        // the deepest group (the longest SMM, the fewest walks) goes second,
        // where its SMM runs beside the walks of the shallowest group
        if (is_static && jobs.size() >= 3) std::rotate(jobs.begin() + 1, jobs.end() - 1, jobs.end());
    }
    for (size_t i = 0; i < jobs.size(); ++i) jobs[i].set = (int)(i % sets);
    // walk filters: per slot set, room for the largest group
    int64_t job_nq_max = 0;
    for (const Job &jb : jobs)
        job_nq_max = std::max<int64_t>(job_nq_max, std::min<int64_t>(jb.gp.pend, jb.gp.p0 + jb.gp.nbat * B) - jb.gp.p0);
    GEER_TRY(g->ws.wfilter.reserve((size_t)sets * std::max<int64_t>(job_nq_max, 1) * kWalkFilterWords *
                                   sizeof(unsigned long long)));
    auto filter_of = [&](int set) {
        return g->ws.wfilter.as<unsigned long long>() + (size_t)set * job_nq_max * kWalkFilterWords;
    };
    const size_t set_vals = (size_t)G * 3 * g->n * kCols, set_words = (size_t)G * 3 * g->n * kBitWords;
    auto view = [&](int set) {
        SlotView v{g->ws.pool.as<char>() + set * set_vals * vs, g->ws.bits.as<uint32_t>() + set * set_words,
                   (size_t)g->n, vs, set * G};
        return v;
    };
    auto meta = [&](int set) { return SlotMeta{g->ws.meta.as<uint64_t>() + set * meta_words, G}; };
    std::vector<std::vector<BatchRec>> recs(sets, std::vector<BatchRec>(G));
    // sB: the AMC stream (a second library stream when there are two slot
    // sets); a captured range runs on sA alone (see below)
    hipStream_t sA = c.stream, sB = sets == 2 ? g->stream2 : c.stream;
    QueryCtx cB = c;
    // restore job i's slots to zero on sA once its walks (on sB) are done, so
    // that the cleanup runs beside the next job's walks instead of before them
    auto cleanup = [&](size_t i) -> geer_status {
        const Job &jb = jobs[i];
        const SlotView v = view(jb.set);
        const SlotMeta m = meta(jb.set);
        if (sB != sA) GEER_HIP(hipStreamWaitEvent(sA, g->ev_clean[jb.set], 0));
        return cleanup_group(g, c, v, m, slot_args(g, v, m, jb.gp), (int)jb.gp.nbat, recs[jb.set]);
    };
    // a fixed AMC plan (captured jobs): the reserved partials, the call's
    // overflow word, and each group's rounds from its largest batch count
    int64_t *sticky = g->ws.misc.as<int64_t>() + kMiscSticky;
    int64_t zcap = 0;
    auto group_rounds = [&](const Job &jb) {
        int r = 1;
        const int64_t pe = std::min<int64_t>(jb.gp.pend, jb.gp.p0 + jb.gp.nbat * B);
        for (int64_t i = jb.gp.p0; i < pe; ++i) r = std::max(r, taus[ord[i]]);
        return r;
    };
    // AMC phase of job i on sB, after its SMM on sA
    auto amc = [&](size_t i, bool fixed) -> geer_status {
        const Job &jb = jobs[i];
        if (sB != sA) GEER_HIP(hipStreamWaitEvent(sB, g->ev_smm[jb.set], 0));
        AmcGroup grp;
        grp.q0 = jb.gp.p0;
        grp.nq = std::min<int64_t>(jb.gp.pend, jb.gp.p0 + jb.gp.nbat * B) - grp.q0;
        grp.pool = view(jb.set).pool;
        grp.value_size = vs;
        grp.filter = filter_of(jb.set);
        if (fixed) {
            grp.fixed_plan = true;
            grp.rounds = group_rounds(jb);
            grp.zpart_cap = zcap;
            grp.sticky = sticky;
        }
        cB.stream = sB;
        GEER_TRY(amc_phase(g, cB, grp, sB, p.walk_ilp));
        if (sB == sA) return cleanup(i);  // one stream: the next job may reuse the slots
        GEER_HIP(hipEventRecord(g->ev_clean[jb.set], sB));
        return GEER_OK;
    };
    // Jobs [j0, j1): the AMC phase of job i - 1 is queued (its chunk bound
    // read first, unless the plan is fixed) before the SMM of job i, so both
    // run at once on the two slot sets; job i - 2's cleanup (same slot set as
    // job i, whose records it reads) comes first.  The last two cleanups
    // also order sA after every walk on sB.
    auto run_jobs = [&](size_t j0, size_t j1, bool fixed) -> geer_status {
        for (size_t i = j0; i <= j1; ++i) {
            if (i >= j0 + 1) GEER_TRY(amc(i - 1, fixed));
            if (i == j1) break;
            const Job &jb = jobs[i];
            if (sB != sA && i >= j0 + 2) GEER_TRY(cleanup(i - 2));
            GEER_TRY(smm_group(g, c, view(jb.set), meta(jb.set), jb.gp, jb.is_static, target.data(), h_s,
                               h_t, ord.data(), col_tile, max_hops, recs[jb.set]));
            GEER_TRY(launch_walk_filter(g, c, jb.gp.p0,
                                        (int)(std::min<int64_t>(jb.gp.pend, jb.gp.p0 + jb.gp.nbat * B) - jb.gp.p0),
                                        filter_of(jb.set), sA));
            if (sB != sA) GEER_HIP(hipEventRecord(g->ev_smm[jb.set], sA));
        }
        if (sB != sA)
            for (size_t i = j1 >= j0 + 2 ? j1 - 2 : j0; i < j1; ++i) GEER_TRY(cleanup(i));
        return GEER_OK;
    };
    size_t n_fixed = 0;  // jobs run by the captured graph
    if (graph_mode)
        while (n_fixed < jobs.size() && jobs[n_fixed].is_static) ++n_fixed;
    if (n_fixed > 0) {
        // reserve every buffer the captured jobs use, then capture them (or
        // replay the graph of an earlier call that derived the same launches)
        zcap = kFixedPlanChunks;
        GEER_TRY(g->ws.zpart.reserve((size_t)zcap * sizeof(double2)));
        GEER_TRY(g->ws.chunk_off.reserve(((size_t)G * B + 1) * sizeof(int64_t)));
        GEER_TRY(reserve_dense(g, vs));
        geer_status aerr = GEER_OK;
        ensure_hop2_acc(g, G, sA, &aerr);
        GEER_TRY(aerr);
        GraphSig sig;
        sig.add(c.nq);
        sig.add(vs);
        sig.add(B);
        sig.add(G);
        sig.add(sets);
        sig.add(col_tile);
        sig.add(n_static);
        sig.add(n_fixed);
        sig.add(max_hops);
        sig.add(meta_words);
        sig.add(zcap);
        sig.add(c.tau);
        sig.add(c.delta);
        sig.add(c.seed);
        sig.add(c.qid_offset);
        sig.add(c.schedule);
        sig.add(c.hop1_implicit);
        sig.add(p.walk_ilp);
        sig.add(sA);
        sig.add(sB);
        const Workspace &w = g->ws;
        for (const DevBuf *b : {&w.pool, &w.bits, &w.part, &w.segbuf, &w.colstat, &w.hpart, &w.qstate,
                                &w.chunk_off, &w.zpart, &w.misc, &w.acc, &w.meta, &w.wfilter})
            sig.add(b->ptr);
        sig.add(w.acc_slots);
        sig.add(w.nq_cap);
        sig.add_n(w.a_dirty.data(), w.a_dirty.size());
        sig.add_n(g->tile_ns, 3);
        for (int64_t i = 0; i < n_static; ++i) {
            const int32_t q = ord[i];
            sig.add(q);
            sig.add(target[q]);
            sig.add(taus[q]);
            sig.add(h_s[q]);
            sig.add(h_t[q]);
        }
        // the host-side state the captured jobs leave behind (slot records,
        // dirty buffers) is what running them leaves: derive it by capturing
        // again whenever the signature differs
        const bool replay = g->gexec && sig.b == g->gsig;
        std::vector<char> dirty_after;
        if (replay) {
            dirty_after = g->gdirty;
        } else {
            if (g->gexec) {
                (void)hipGraphExecDestroy(g->gexec);
                g->gexec = nullptr;
                g->gsig.clear();
            }
            // The captured range runs on sA alone (SMM, AMC and cleanup of
            // each group in turn): a graph with parallel branches, captured
            // again after an earlier capture and later destroyed, at times
            // kept the device memory its kernels addressed from being
            // returned when freed (measured on MI355X, ROCm 7.2); linear
            // graphs never did.
            const hipStream_t sB_direct = sB;
            sB = sA;
            geer_status st = GEER_OK;
            const hipError_t be = hipStreamBeginCapture(sA, hipStreamCaptureModeThreadLocal);
            const bool prof_on = g->prof.on;
            if (be == hipSuccess) {
                g->prof.on = false;
                t_capturing = true;
                st = launch_zero(g, sticky, 2 * sizeof(int64_t), sA);
                if (st == GEER_OK) st = run_jobs(0, n_fixed, true);
                t_capturing = false;
                g->prof.on = prof_on;
            }
            hipGraph_t graph = nullptr;
            const hipError_t ce = be == hipSuccess ? hipStreamEndCapture(sA, &graph) : be;
            sB = sB_direct;
            if (st != GEER_OK || ce != hipSuccess) {
                if (graph) (void)hipGraphDestroy(graph);
                (void)hipGetLastError();
                return st != GEER_OK ? st : fail(GEER_E_DEVICE, std::string("hipStreamEndCapture: ") +
                                                                      hipGetErrorString(ce));
            }
            const hipError_t ie = hipGraphInstantiate(&g->gexec, graph, nullptr, nullptr, 0);
            (void)hipGraphDestroy(graph);
            if (ie != hipSuccess) {
                g->gexec = nullptr;
                return fail(GEER_E_DEVICE, std::string("hipGraphInstantiate: ") + hipGetErrorString(ie));
            }
            g->gsig = std::move(sig.b);
            g->gdirty = w.a_dirty;
        }
        int tok = prof_begin(g, sA);
        GEER_HIP(hipGraphLaunch(g->gexec, sA));
        prof_end(g, tok, PK_GRAPH, 0.0, 1.0, sA);
        if (replay) g->ws.a_dirty = dirty_after;
    }
    GEER_TRY(run_jobs(n_fixed, jobs.size(), false));
    if (n_fixed > 0) {
        int64_t flag = 0;
        GEER_HIP(hipMemcpyAsync(&flag, sticky, sizeof(flag), hipMemcpyDeviceToHost, sA));
        GEER_HIP(hipStreamSynchronize(sA));
        if (flag & 2) return fail(GEER_E_INVALID_ARG, "AMC batch exceeds 2^32 walk pairs for a query");
        if (flag & 1)
            return fail(GEER_E_OOM, "an AMC round of the captured plan needs more than " +
                                        std::to_string(zcap) + " chunk partials");
    }
    g->ws.in_use = false;
    return GEER_OK;
}

static hipStream_t pick_stream(geer_graph *g, const geer_params &p)
{
    return p.stream ? (hipStream_t)p.stream : g->stream;
}

}  // namespace geer

using namespace geer;

extern "C" {

geer_status geer_params_default(geer_params *p)
{
    if (!p) return fail(GEER_E_INVALID_ARG, "params is NULL");
    std::memset(p, 0, sizeof(*p));
    p->delta = 0.01;
    p->tau = 5;
    p->schedule = GEER_SCHEDULE_GREEDY;
    return GEER_OK;
}

geer_status geer_query(geer_graph *g, int64_t nq, const int32_t *s, const int32_t *t,
                       const double *eps, const geer_params *params, double *r_out,
                       geer_query_stats *stats)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (nq < 0) return fail(GEER_E_INVALID_ARG, "nq must be >= 0");
    if (nq > 0 && (!s || !t || !eps || !r_out)) return fail(GEER_E_INVALID_ARG, "NULL array");
    geer_params p;
    if (params) p = *params;
    else geer_params_default(&p);
    GEER_TRY(check_params(p));
    if (!g->has_lambda) return fail(GEER_E_NO_LAMBDA, "lambda has not been set");
    if (p.schedule == GEER_SCHEDULE_FIXED && nq > 0 && !p.fixed_ell_b)
        return fail(GEER_E_INVALID_ARG, "FIXED schedule needs fixed_ell_b");
    for (int64_t i = 0; i < nq; ++i) {
        if (s[i] < 0 || s[i] >= g->n || t[i] < 0 || t[i] >= g->n)
            return fail(GEER_E_INVALID_ARG, "query " + std::to_string(i) + ": node out of range");
        if (!(eps[i] > 0.0) || std::isinf(eps[i]))
            return fail(GEER_E_INVALID_ARG, "query " + std::to_string(i) + ": eps must be > 0 and finite");
    }
    if (nq == 0) return GEER_OK;
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, p);
    QueryCtx c;
    GEER_TRY(ensure_qstate(g, nq, &c.qs));
    c.nq = nq;
    c.lambda = g->lambda;
    c.delta = p.delta;
    c.tau = p.tau;
    c.schedule = p.schedule;
    c.seed = p.seed;
    c.qid_offset = p.qid_offset;
    c.ell_rule = (p.flags & GEER_FLAG_PENG_ELL) ? 1 : 0;
    // stage inputs / outputs
    const size_t io_bytes = (size_t)nq * (sizeof(double) + sizeof(int32_t) + sizeof(geer_query_stats)) + 256;
    GEER_TRY(g->ws.io.reserve(io_bytes));
    double *d_r = g->ws.io.as<double>();
    int32_t *d_fixed = reinterpret_cast<int32_t *>(d_r + nq);
    geer_query_stats *d_stats = reinterpret_cast<geer_query_stats *>(
        (char *)g->ws.io.ptr + (((size_t)nq * (sizeof(double) + sizeof(int32_t)) + 15) / 16) * 16);
    GEER_HIP(hipMemcpyAsync(c.qs.s, s, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.t, t, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.eps, eps, nq * sizeof(double), hipMemcpyHostToDevice, st));
    if (p.schedule == GEER_SCHEDULE_FIXED)
        GEER_HIP(hipMemcpyAsync(d_fixed, p.fixed_ell_b, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    double min_eps = eps[0];
    for (int64_t i = 1; i < nq; ++i) min_eps = std::min(min_eps, eps[i]);
    c.stream = st;
    GEER_TRY(run_queries(g, c, p, d_fixed, min_eps, s, t));
    GEER_TRY(launch_finalize(g, c, d_r, stats ? d_stats : nullptr, st));
    GEER_HIP(hipMemcpyAsync(r_out, d_r, nq * sizeof(double), hipMemcpyDeviceToHost, st));
    if (stats)
        GEER_HIP(hipMemcpyAsync(stats, d_stats, nq * sizeof(geer_query_stats), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    return GEER_OK;
}

geer_status geer_query_device(geer_graph *g, int64_t nq, const int32_t *d_s, const int32_t *d_t,
                              const double *d_eps, const geer_params *params, double *d_r_out,
                              geer_query_stats *d_stats)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (nq < 0) return fail(GEER_E_INVALID_ARG, "nq must be >= 0");
    if (nq > 0 && (!d_s || !d_t || !d_eps || !d_r_out)) return fail(GEER_E_INVALID_ARG, "NULL array");
    geer_params p;
    if (params) p = *params;
    else geer_params_default(&p);
    GEER_TRY(check_params(p));
    if (!g->has_lambda) return fail(GEER_E_NO_LAMBDA, "lambda has not been set");
    if (p.schedule == GEER_SCHEDULE_FIXED && nq > 0 && !p.fixed_ell_b)
        return fail(GEER_E_INVALID_ARG, "FIXED schedule needs fixed_ell_b");
    if (nq == 0) return GEER_OK;
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = pick_stream(g, p);
    QueryCtx c;
    GEER_TRY(ensure_qstate(g, nq, &c.qs));
    c.nq = nq;
    c.lambda = g->lambda;
    c.delta = p.delta;
    c.tau = p.tau;
    c.schedule = p.schedule;
    c.seed = p.seed;
    c.qid_offset = p.qid_offset;
    c.ell_rule = (p.flags & GEER_FLAG_PENG_ELL) ? 1 : 0;
    if (!p.stream) {
        // no stream given: order after all work already queued on the legacy
        // default stream (where the caller's inputs were most likely produced)
        hipEvent_t ev;
        GEER_HIP(hipEventCreateWithFlags(&ev, hipEventDisableTiming));
        GEER_HIP(hipEventRecord(ev, nullptr));
        GEER_HIP(hipStreamWaitEvent(st, ev, 0));
        GEER_HIP(hipEventDestroy(ev));
    }
    GEER_TRY(g->ws.io.reserve((size_t)nq * sizeof(int32_t) + 256));
    int32_t *d_fixed = g->ws.io.as<int32_t>();
    GEER_HIP(hipMemcpyAsync(c.qs.s, d_s, nq * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.t, d_t, nq * sizeof(int32_t), hipMemcpyDeviceToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.eps, d_eps, nq * sizeof(double), hipMemcpyDeviceToDevice, st));
    if (p.schedule == GEER_SCHEDULE_FIXED)
        GEER_HIP(hipMemcpyAsync(d_fixed, p.fixed_ell_b, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    std::vector<double> heps(nq);
    std::vector<int32_t> hs(nq), ht(nq);
    GEER_HIP(hipMemcpyAsync(heps.data(), d_eps, nq * sizeof(double), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipMemcpyAsync(hs.data(), d_s, nq * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipMemcpyAsync(ht.data(), d_t, nq * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    double min_eps = 1e300;
    for (double e : heps)
        if (e > 0.0 && e < min_eps) min_eps = e;
    // out-of-range ids are reported after the run; plan with clamped copies
    for (int64_t i = 0; i < nq; ++i) {
        hs[i] = std::min(std::max(hs[i], 0), g->n - 1);
        ht[i] = std::min(std::max(ht[i], 0), g->n - 1);
    }
    c.stream = st;
    GEER_TRY(run_queries(g, c, p, d_fixed, min_eps, hs.data(), ht.data()));
    GEER_TRY(launch_finalize(g, c, d_r_out, d_stats, st));
    GEER_HIP(hipStreamSynchronize(st));
    // invalid entries were turned into NaN results by the init kernel
    std::vector<int32_t> stop(nq);
    GEER_HIP(hipMemcpy(stop.data(), c.qs.stop, nq * sizeof(int32_t), hipMemcpyDeviceToHost));
    for (int64_t i = 0; i < nq; ++i)
        if (stop[i] < 0)
            return fail(GEER_E_INVALID_ARG, "query " + std::to_string(i) + ": node id or eps invalid");
    return GEER_OK;
}

geer_status geer_smm(geer_graph *g, int32_t nq, const int32_t *s, const int32_t *t, int32_t hops,
                     uint32_t flags, int32_t col_tile, void *vec_out, double *rb_out,
                     double *top2_out, int64_t *supp_out)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (nq < 1 || nq > kMaxPairs) return fail(GEER_E_INVALID_ARG, "nq must be in 1..64");
    if (!s || !t || !vec_out) return fail(GEER_E_INVALID_ARG, "NULL array");
    if (hops < 0) return fail(GEER_E_INVALID_ARG, "hops must be >= 0");
    if (col_tile != 0 && col_tile != 32 && col_tile != 64 && col_tile != 128)
        return fail(GEER_E_INVALID_ARG, "col_tile must be 0, 32, 64 or 128");
    for (int i = 0; i < nq; ++i)
        if (s[i] < 0 || s[i] >= g->n || t[i] < 0 || t[i] >= g->n)
            return fail(GEER_E_INVALID_ARG, "node out of range");
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    const int vs = (flags & GEER_FLAG_FP64_VECTORS) ? 8 : 4;
    QueryCtx c;
    GEER_TRY(ensure_qstate(g, nq, &c.qs));
    c.nq = nq;
    c.lambda = 0.5;
    c.delta = 0.01;
    c.tau = 5;
    c.schedule = GEER_SCHEDULE_FIXED;
    c.seed = 0;
    c.qid_offset = 0;
    begin_slot_use(g);
    GEER_TRY(ensure_slots(g, std::max(1, g->ws.slots), vs));
    std::vector<double> ones(nq, 1.0);
    GEER_HIP(hipMemcpyAsync(c.qs.s, s, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.t, t, nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(c.qs.eps, ones.data(), nq * sizeof(double), hipMemcpyHostToDevice, st));
    GEER_TRY(launch_init_queries(g, c, nullptr, hops, st));
    SlotView sv{g->ws.pool.as<char>(), g->ws.bits.as<uint32_t>(), (size_t)g->n, vs};
    const int tile = col_tile ? -col_tile : default_col_tile(g, vs);
    c.stream = st;
    std::vector<int32_t> ord(nq), target(nq, hops);
    for (int i = 0; i < nq; ++i) ord[i] = i;
    GEER_HIP(hipMemcpyAsync(c.qs.ord, ord.data(), nq * sizeof(int32_t), hipMemcpyHostToDevice, st));
    const int G1 = std::max(1, g->ws.slots);
    GEER_TRY(g->ws.meta.reserve((6 * (size_t)G1 + (size_t)G1 * (hops + 2)) * 8 + 64));
    SlotMeta sm{g->ws.meta.as<uint64_t>(), G1};
    std::vector<BatchRec> recs(1);
    GroupPlan gp;
    gp.p0 = 0;
    gp.nbat = 1;
    gp.pend = nq;
    gp.B = nq;
    if (hops > 0)
        GEER_TRY(smm_group(g, c, sv, sm, gp, true, target.data(), s, t, ord.data(), tile, hops, recs));
    GEER_HIP(hipStreamSynchronize(st));
    const size_t n = (size_t)g->n;
    if (hops == 0) {
        // the hop-0 vectors are e_s and e_t
        std::memset(vec_out, 0, n * 2 * nq * vs);
        for (int j = 0; j < nq; ++j) {
            if (vs == 4) {
                ((float *)vec_out)[(size_t)s[j] * 2 * nq + 2 * j] = 1.0f;
                ((float *)vec_out)[(size_t)t[j] * 2 * nq + 2 * j + 1] = 1.0f;
            } else {
                ((double *)vec_out)[(size_t)s[j] * 2 * nq + 2 * j] = 1.0;
                ((double *)vec_out)[(size_t)t[j] * 2 * nq + 2 * j + 1] = 1.0;
            }
        }
    } else {
        const int which = hops == 1 ? 0 : (hops % 2 == 0 ? 1 : 2);
        GEER_HIP(hipMemcpy2D(vec_out, (size_t)2 * nq * vs, sv.buf(0, which), (size_t)kCols * vs,
                             (size_t)2 * nq * vs, n, hipMemcpyDeviceToHost));
    }
    if (rb_out) {
        std::vector<double> rb(nq);
        GEER_HIP(hipMemcpy(rb.data(), c.qs.rb, nq * sizeof(double), hipMemcpyDeviceToHost));
        for (int j = 0; j < nq; ++j) rb_out[j] = s[j] == t[j] ? 0.0 : rb[j];
    }
    if (top2_out || supp_out) {
        std::vector<double> cs(2 * kCols);
        std::vector<int64_t> sd(kCols);
        if (hops > 0) {
            GEER_HIP(hipMemcpy(cs.data(), g->ws.colstat.ptr, 2 * kCols * sizeof(double), hipMemcpyDeviceToHost));
            GEER_HIP(hipMemcpy(sd.data(), (char *)g->ws.colstat.ptr + 2 * kCols * sizeof(double),
                               kCols * sizeof(int64_t), hipMemcpyDeviceToHost));
        }
        for (int j = 0; j < nq; ++j) {
            for (int side = 0; side < 2; ++side) {
                const int c2 = 2 * j + side;
                double m1 = 1.0, m2 = 0.0;
                int64_t d = 0;
                if (hops > 0) {
                    m1 = cs[c2];
                    m2 = cs[kCols + c2];
                    d = sd[c2];
                } else {
                    int32_t u = side ? t[j] : s[j];
                    int32_t rp[2];
                    GEER_HIP(hipMemcpy(rp, g->d_row_ptr + u, 2 * sizeof(int32_t), hipMemcpyDeviceToHost));
                    d = rp[1] - rp[0];
                }
                if (top2_out) {
                    top2_out[4 * j + 2 * side] = m1;
                    top2_out[4 * j + 2 * side + 1] = m2;
                }
                if (supp_out) supp_out[2 * j + side] = d;
            }
        }
    }
    // restore the sparse buffers to zero
    if (hops > 0) {
        GEER_TRY(cleanup_group(g, c, sv, sm, slot_args(g, sv, sm, gp), 1, recs));
        GEER_HIP(hipStreamSynchronize(st));
    }
    g->ws.in_use = false;
    return GEER_OK;
}

geer_status geer_walk_traces(geer_graph *g, int32_t nw, const int32_t *start, const uint32_t *q,
                             const uint32_t *batch, const uint32_t *k, const uint32_t *side,
                             int32_t lf, uint64_t seed, int32_t *trace_out)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (nw < 0 || lf < 0) return fail(GEER_E_INVALID_ARG, "negative size");
    if (nw == 0 || lf == 0) return GEER_OK;
    if (!start || !q || !batch || !k || !side || !trace_out)
        return fail(GEER_E_INVALID_ARG, "NULL array");
    for (int32_t i = 0; i < nw; ++i) {
        if (start[i] < 0 || start[i] >= g->n) return fail(GEER_E_INVALID_ARG, "start out of range");
        if (side[i] > 1) return fail(GEER_E_INVALID_ARG, "side must be 0 or 1");
        if (batch[i] >= (1u << 31)) return fail(GEER_E_INVALID_ARG, "batch too large");
    }
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    const size_t bytes = (size_t)nw * (sizeof(int32_t) + 4 * sizeof(uint32_t)) + (size_t)nw * lf * sizeof(int32_t) + 256;
    GEER_TRY(g->ws.io.reserve(bytes));
    int32_t *d_start = g->ws.io.as<int32_t>();
    uint32_t *d_q = reinterpret_cast<uint32_t *>(d_start + nw);
    uint32_t *d_b = d_q + nw;
    uint32_t *d_k = d_b + nw;
    uint32_t *d_side = d_k + nw;
    int32_t *d_trace = reinterpret_cast<int32_t *>(d_side + nw);
    GEER_HIP(hipMemcpyAsync(d_start, start, nw * sizeof(int32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_q, q, nw * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_b, batch, nw * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_k, k, nw * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    GEER_HIP(hipMemcpyAsync(d_side, side, nw * sizeof(uint32_t), hipMemcpyHostToDevice, st));
    GEER_TRY(launch_walk_traces(g, nw, d_start, d_q, d_b, d_k, d_side, lf, seed, d_trace, st));
    GEER_HIP(hipMemcpyAsync(trace_out, d_trace, (size_t)nw * lf * sizeof(int32_t), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    return GEER_OK;
}

}  // extern "C"


extern "C" geer_status geer_amc(geer_graph *g, int32_t s, int32_t t, const double *x,
                                const double *y, double eps, int32_t lf, int32_t tau,
                                double delta, uint64_t seed, uint32_t q, uint32_t flags,
                                double *rf_out, geer_query_stats *stats)
{
    if (!g) return fail(GEER_E_INVALID_ARG, "graph is NULL");
    if (!x || !y || !rf_out) return fail(GEER_E_INVALID_ARG, "NULL array");
    if (s < 0 || s >= g->n || t < 0 || t >= g->n) return fail(GEER_E_INVALID_ARG, "node out of range");
    if (!(eps > 0.0) || std::isinf(eps)) return fail(GEER_E_INVALID_ARG, "eps must be > 0");
    if (lf < 0) return fail(GEER_E_INVALID_ARG, "lf must be >= 0");
    if (tau < 1 || tau > 30) return fail(GEER_E_INVALID_ARG, "tau must be in 1..30");
    if (!(delta > 0.0 && delta < 1.0)) return fail(GEER_E_INVALID_ARG, "delta must be in (0,1)");
    const int32_t n = g->n;
    for (int32_t v = 0; v < n; ++v)
        if (!(x[v] >= 0.0) || !(y[v] >= 0.0) || std::isinf(x[v]) || std::isinf(y[v]))
            return fail(GEER_E_INVALID_ARG, "vectors must be finite and non-negative");
    GEER_HIP(hipSetDevice(g->device));
    hipStream_t st = g->stream;
    const int vs = (flags & GEER_FLAG_FP64_VECTORS) ? 8 : 4;
    QueryCtx c;
    GEER_TRY(ensure_qstate(g, 1, &c.qs));
    c.nq = 1;
    c.lambda = 0.5;
    c.delta = delta;
    c.tau = tau;
    c.schedule = GEER_SCHEDULE_FIXED;
    c.seed = seed;
    c.qid_offset = (int64_t)q;
    GEER_TRY(ensure_slots(g, std::max(1, g->ws.slots), vs));
    SlotView sv{g->ws.pool.as<char>(), g->ws.bits.as<uint32_t>(), (size_t)n, vs};
    // interleave (x, y) into columns 0, 1 of slot 0's A buffer
    std::vector<char> host((size_t)n * 2 * vs);
    for (int32_t v = 0; v < n; ++v) {
        if (vs == 4) {
            ((float *)host.data())[2 * (size_t)v] = (float)x[v];
            ((float *)host.data())[2 * (size_t)v + 1] = (float)y[v];
        } else {
            ((double *)host.data())[2 * (size_t)v] = x[v];
            ((double *)host.data())[2 * (size_t)v + 1] = y[v];
        }
    }
    g->ws.a_dirty[0] = 1;  // A holds dense caller vectors (zeroed in full before a sparse use)
    GEER_HIP(hipMemcpy2D(sv.buf(0, 1), (size_t)kCols * vs, host.data(), (size_t)2 * vs, (size_t)2 * vs,
                         (size_t)n, hipMemcpyHostToDevice));
    c.stream = st;
    double *cs_m1 = g->ws.colstat.as<double>();
    GEER_TRY(launch_column_top2(g, sv.buf(0, 1), 2, kCols, vs, cs_m1, cs_m1 + kCols, st));
    GEER_TRY(launch_amc_setup(g, c.qs, s, t, lf, eps, tau, delta, sv.elem_off(0, 1), cs_m1,
                              cs_m1 + kCols, st));
    AmcGroup grp;
    grp.q0 = 0;
    grp.nq = 1;
    grp.pool = sv.pool;
    grp.value_size = vs;
    // the walk counter uses q + qid_offset with q = 0 here, so qid_offset = q
    GEER_TRY(amc_phase(g, c, grp, st, 0));
    GEER_TRY(g->ws.io.reserve(sizeof(double) + sizeof(geer_query_stats) + 64));
    double *d_r = g->ws.io.as<double>();
    geer_query_stats *d_st = reinterpret_cast<geer_query_stats *>((char *)g->ws.io.ptr + 16);
    GEER_TRY(launch_finalize(g, c, d_r, d_st, st));
    geer_query_stats hs;
    GEER_HIP(hipMemcpyAsync(&hs, d_st, sizeof(hs), hipMemcpyDeviceToHost, st));
    GEER_HIP(hipStreamSynchronize(st));
    *rf_out = hs.r_f;
    if (stats) {
        *stats = hs;
        stats->ell = -1;
        stats->ell_b = -1;
    }
    return GEER_OK;
}
