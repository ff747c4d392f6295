// Internal declarations of the MI355X GEER library (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/geer.h"

// ----------------------------------------------------------------------------
// Error plumbing
// ----------------------------------------------------------------------------

namespace geer {

void set_error(const std::string &msg);
geer_status fail(geer_status st, const std::string &msg);

#define GEER_HIP(call)                                                                 \
    do {                                                                               \
        hipError_t e_ = (call);                                                        \
        if (e_ != hipSuccess)                                                          \
            return ::geer::fail(GEER_E_DEVICE, std::string(#call) + ": " +             \
                                                   hipGetErrorString(e_));             \
    } while (0)

#define GEER_TRY(expr)                                                                 \
    do {                                                                               \
        geer_status s_ = (expr);                                                       \
        if (s_ != GEER_OK) return s_;                                                  \
    } while (0)

// ----------------------------------------------------------------------------
// Fixed layout constants
// ----------------------------------------------------------------------------

constexpr int kCols = 128;            // vector columns per SMM batch slot (64 pairs x {s, t})
constexpr int kMaxPairs = kCols / 2;  // pairs per SMM batch
constexpr int kBitWords = kCols / 32; // support bitmask words per node
constexpr int kSegNnz = 256;          // rows longer than this are split into segments
constexpr int kPairsPerChunk = 32;    // walk pairs per wavefront work item (64 lanes)
constexpr int kLearnedTauMax = 8;     // largest AMC batch count the learned schedule picks
// misc scratch layout (int64 words): [8] AMC chunk total of the current
// round, [10, 12) walk steps of the round (when not profiled), [12, 15) AMC
// chunk bound, overflow flag and largest batch count of the group
constexpr int kMiscWords = 16;
constexpr int kMiscSticky = 16;  // [16, 18): overflow word of a captured call (workspace misc only)
// chunk partials reserved for a captured call's AMC rounds (2^24 x 16 B =
// 256 MB: about 5.4e8 walk pairs in one round of one group)
constexpr int64_t kFixedPlanChunks = int64_t(1) << 24;

// ----------------------------------------------------------------------------
// Device-resident growable buffer
// ----------------------------------------------------------------------------

// Set while a call's launch sequence is being captured into a hipGraph: a
// buffer that would have to grow then fails instead of allocating (every
// buffer the captured sequence uses is reserved before capture begins).
extern thread_local bool t_capturing;

struct DevBuf {
    void *ptr = nullptr;
    size_t bytes = 0;
    // a captured launch graph whose kernels may address this buffer: it is
    // destroyed before the buffer is freed (memory freed while an executable
    // graph that was launched more than once still refers to it was not
    // returned to the device)
    hipGraphExec_t *dependent = nullptr;
    geer_status reserve(size_t want);
    void release();
    template <class T> T *as() const { return static_cast<T *>(ptr); }
};

// ----------------------------------------------------------------------------
// Per-query device state (structure of arrays, one allocation)
// ----------------------------------------------------------------------------

struct QState {
    int32_t *s, *t, *ell, *lb, *lb_target, *lf, *batches, *stop, *active_smm, *active_amc,
        *fallback, *tau_q;
    int32_t *ord;  // batch position -> query index (batches take consecutive positions)
    int32_t *h1w;  // 1 while the pair's two hop-1 columns hold scattered entries
    int64_t *eta1, *walk_pairs, *supp_sum, *vec_off;
    double *eps, *rb, *psi, *eta_star, *zsum, *z2sum, *var, *f, *rf, *r;
};

struct Workspace {
    DevBuf pool;      // SMM vectors: slots x {H1, A, B} x n x kCols values
    DevBuf bits;      // structural supports: slots x {H1, A, B} x n x kBitWords
    DevBuf part;      // per-block column statistics (max1, max2 as double; degree sums)
    DevBuf segbuf;    // heavy-row segment partial sums (values + bits)
    DevBuf colstat;   // per slot: per-column reduced statistics of the current hop
    DevBuf hpart;     // per slot: hop-2 partial column statistics (kPushSplitMax rows)
    DevBuf qstate;    // QState arrays
    DevBuf chunk_off; // AMC: chunk prefix sums per group query
    DevBuf zpart;     // AMC: per-chunk (sum Z, sum Z^2)
    DevBuf misc;      // small scalars (active masks, totals)
    DevBuf io;        // staging for host inputs/outputs
    DevBuf acc;       // sparse hop 2: per slot n x kCols fixed-point accumulators (kept all zero)
    DevBuf meta;      // per-slot masks (active, hop-2 cleanup, hop-2 paths, static levels)
    DevBuf feat;      // learned scheduler: per-pair features
    DevBuf wfilter;   // walk filters: per slot set, per group position
    int acc_slots = 0;          // slots of all-zero accumulators held in acc
    bool in_use = false;        // a call holds entries in the slot buffers (set until it restores them)
    std::vector<char> a_dirty;  // per slot: buffer A was written by a dense hop
    int slots = 0;
    int value_size = 0;
    int64_t nq_cap = 0;
};

// Event timing of kernel launches (enabled by geer_profile_enable).
enum ProfKind {
    PK_HOP_LIGHT = 0,
    PK_HOP_SEGMENTS,
    PK_HOP_HEAVY_FIN,
    PK_HOP1,
    PK_COLSTAT,
    PK_EPILOGUE,
    PK_WALK,
    PK_AMC_PLAN,
    PK_AMC_STOP,
    PK_FEATURES,
    PK_MLP,
    PK_HOP2_SPARSE,
    PK_HOP2_LDS,
    PK_DENSE_HOP,
    PK_GRAPH,  // one launch of a captured call (all of its kernels)
    PK_COUNT
};

struct ProfRec {
    int kind;
    hipEvent_t a, b;
    double bytes, units;
    // counted records: bytes = per_unit * c0 + per_unit2 * c1 and units = c0,
    // with (c0, c1) written on the device into counter slot `counter`
    int counter = -1;
    double per_unit = 0.0, per_unit2 = 0.0;
};

constexpr int kProfCounters = 4096;  // device counter pairs between two flushes

struct Profiler {
    bool on = false;
    int64_t *d_counters = nullptr;  // kProfCounters x 2 int64
    int n_counters = 0;
    std::vector<ProfRec> recs;
    std::vector<hipEvent_t> spare;
    int64_t launches[PK_COUNT] = {};
    double ms[PK_COUNT] = {}, bytes[PK_COUNT] = {}, units[PK_COUNT] = {};
};

}  // namespace geer

// ----------------------------------------------------------------------------
// The opaque graph handle
// ----------------------------------------------------------------------------

struct geer_graph {
    int device = 0;
    int32_t n = 0;
    int64_t nnz = 0;
    int32_t max_deg = 0;
    double lambda = -1.0;
    bool has_lambda = false;
    hipStream_t stream = nullptr;
    // AMC phases run on stream2 while the next group's SMM runs on the query
    // stream; the events order the two slot sets between them
    hipStream_t stream2 = nullptr;
    hipEvent_t ev_smm[2] = {nullptr, nullptr}, ev_clean[2] = {nullptr, nullptr};
    // pinned host staging of the per-pair depth read and the batch order
    // upload; pin_ev follows the last copy that reads it
    char *h_pin = nullptr;
    size_t h_pin_bytes = 0;
    hipEvent_t pin_ev = nullptr;
    int num_cus = 0;
    // CSR on device
    int32_t *d_row_ptr = nullptr;
    int32_t *d_col_idx = nullptr;
    float *d_inv_deg_f = nullptr;
    double *d_inv_deg_d = nullptr;
    // walk records, one per CSR entry e with v = col_idx[e], carrying v, its
    // row start b = row_ptr[v] and degree d, so that a walk step reads one
    // record instead of col_idx and row_ptr: 8 bytes packed as
    // v | b << rec_sb | d << rec_sd when the bit widths fit, else int4 {v, b, d, 0}
    void *d_walk_rec = nullptr;
    int walk_rec_bytes = 16;
    bool wide_records = false;             // GEER_GRAPH_WIDE_WALK_RECORDS
    int rec_sb = 0, rec_sd = 0;
    // SpMM work decomposition: light rows (degree <= kSegNnz) sorted by
    // degree descending, heavy rows split into segments of <= kSegNnz entries
    int32_t *d_light_rows = nullptr;
    int32_t n_light = 0;
    int32_t *d_heavy_rows = nullptr;
    int32_t *d_heavy_seg_start = nullptr;  // [n_heavy + 1] first segment of each heavy row
    int32_t n_heavy = 0;
    int32_t *d_seg_begin = nullptr;        // [n_seg] first CSR entry of each segment
    int32_t *d_seg_end = nullptr;          // [n_seg] one past the last entry
    int32_t n_seg = 0;
    int64_t nnz_heavy = 0;                 // CSR entries in heavy rows
    int fx_shift = 40;                     // fixed-point scale 2^F of the sparse hop
    std::vector<int32_t> h_row_ptr;        // host copy of the row offsets
    int64_t *d_nbr_work = nullptr;         // per node: sum of neighbour degrees
    int32_t *d_min_nbr_deg = nullptr;      // per node: smallest neighbour degree
    int32_t *d_nbr_deg2 = nullptr;         // per node: second smallest (repeats counted; 0 if degree 1)
    double rho2 = 6.0, rhod = 1e6;         // cost ratios (learned-scheduler features)
    int tuned_col_tile = 0;                // autotuner's SpMM column tile (0: not tuned)
    double tile_ns[3] = {0, 0, 0};         // measured time of one tile launch at 32/64/128 columns
    std::vector<int64_t> h_nbr_work;       // sum of neighbour degrees (= sparse hop-2 work)
    // captured launch sequence of the last GEER_FLAG_GRAPH_LAUNCH call and
    // everything its kernels' arguments were derived from (replayed when a
    // later call derives the same)
    hipGraphExec_t gexec = nullptr;
    std::vector<unsigned char> gsig;
    std::vector<char> gdirty;              // Workspace::a_dirty after the captured jobs
    geer::Workspace ws;
    geer::Profiler prof;
};

// ----------------------------------------------------------------------------
// Philox4x32-10 (Salmon, Moraes, Dror, Shaw, SC'11) and the walk sampler.
// Shared by every kernel that draws a walk so that traces and AMC walks are
// the same function of (seed, q, batch, k, side, step).
// ----------------------------------------------------------------------------

namespace geer {

__device__ __forceinline__ uint4 philox4x32_10(uint4 c, uint32_t k0, uint32_t k1)
{
#pragma unroll
    for (int r = 0; r < 10; ++r) {
        const uint32_t m0 = 0xD2511F53u, m1 = 0xCD9E8D57u;
        uint32_t hi0 = __umulhi(m0, c.x), lo0 = m0 * c.x;
        uint32_t hi1 = __umulhi(m1, c.z), lo1 = m1 * c.z;
        c = make_uint4(hi1 ^ c.y ^ k0, lo1, hi0 ^ c.w ^ k1, lo0);
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    return c;
}

__device__ __forceinline__ uint32_t pick_word(const uint4 &r, uint32_t i)
{
    return i == 0 ? r.x : (i == 1 ? r.y : (i == 2 ? r.z : r.w));
}

// One step of a walk: the next node is row u's (draw mod d(u))-th CSR entry.
__device__ __forceinline__ int32_t walk_next(const int32_t *__restrict__ row_ptr,
                                             const int32_t *__restrict__ col_idx, int32_t u,
                                             uint32_t draw)
{
    int32_t b = row_ptr[u];
    uint32_t d = (uint32_t)(row_ptr[u + 1] - b);
    return col_idx[b + (int32_t)(draw % d)];
}

// ----------------------------------------------------------------------------
// Scalar formulas (FP64), same readings as documented in the design notes.
// ----------------------------------------------------------------------------

// Eq. (ell), Theorem 3.1, clamped at 0.
__host__ __device__ inline int32_t ell_of(double ds, double dt, double eps, double lambda)
{
    if (!(lambda > 0.0)) return 0;
    double v = log((2.0 / ds + 2.0 / dt) / (eps * (1.0 - lambda))) / log(1.0 / lambda) - 1.0;
    double c = ceil(v);
    return c < 0.0 ? 0 : (int32_t)c;
}

// Eq. (old-ell): Peng et al.'s pair-independent length, log(4 / (eps (1 - lambda)))
// / log(1 / lambda) - 1, rounded up and clamped at 0 (kept as a variant).
__host__ __device__ inline int32_t ell_peng_of(double eps, double lambda)
{
    if (!(lambda > 0.0)) return 0;
    const double v = log(4.0 / (eps * (1.0 - lambda))) / log(1.0 / lambda) - 1.0;
    const double c = ceil(v);
    return c < 0.0 ? 0 : (int32_t)c;
}

// Eq. (Delta-st).
__host__ __device__ inline double psi_of(int32_t lf, double m1s, double m2s, double m1t,
                                         double m2t, double ids, double idt)
{
    double up = (double)((lf + 1) / 2), dn = (double)(lf / 2);
    return 2.0 * up * (m1s * ids + m1t * idt) + 2.0 * dn * (m2s * ids + m2t * idt);
}

// Eq. (etas-star).
__host__ __device__ inline double eta_star_of(double psi, double eps, int32_t tau, double delta)
{
    return 2.0 * psi * psi * log(2.0 * (double)tau / delta) / (eps * eps);
}

// First AMC batch: ceil(eta* / 2^(tau-1)).
__host__ __device__ inline int64_t eta1_of(double eta_star, int32_t tau)
{
    double v = ceil(eta_star / ldexp(1.0, tau - 1));
    return v <= 0.0 ? 0 : (int64_t)v;
}

// Eq. (fx), empirical Bernstein half-width.
__host__ __device__ inline double bernstein_of(double nz, double var, double psi, double delta)
{
    double lg = log(3.0 / delta);
    return sqrt(2.0 * var * lg / nz) + 3.0 * psi * lg / nz;
}

// ----------------------------------------------------------------------------
// Kernel launchers (defined in smm.hip / amc.hip)
// ----------------------------------------------------------------------------

// Largest row (of s or t) for which the walk kernel evaluates the one-hop
// vectors from the graph instead of reading the vector buffer: on N(s) the
// hop-1 vector is 1/d(u), elsewhere 0, so membership in the (LDS-resident)
// sorted row of s gives the same value as the random read of the buffer.
constexpr int32_t kMemberRowMax = 256;

// Walk filters: a blocked Bloom filter (1024 words of 64 bits, three bits per
// node in one word) of supp(x) U supp(y) for each pair that walks over
// vectors read from the batch slots with a support small enough to filter:
// depth 2, or depth 1 with a row of s or t longer than kMemberRowMax.  A walk
// step whose node is not in the filter reads no vector values (both are
// exactly zero off the supports); a Bloom filter has no false negatives.
// 8 KB per pair: 4 KB and 16 KB filters, and two bits per node, measured
// within 2% of it on the 1M-node Chung-Lu workload
constexpr int kWalkFilterLog2 = 10;
constexpr int kWalkFilterWords = 1 << kWalkFilterLog2;
__host__ __device__ __forceinline__ bool walk_filtered(int64_t voff, int32_t lb, int32_t ds, int32_t dt)
{
    return voff >= 0 && (lb == 2 || (lb == 1 && (ds > kMemberRowMax || dt > kMemberRowMax)));
}
__device__ __forceinline__ uint32_t walk_filter_word(int32_t v)
{
    return ((uint32_t)v * 0x9E3779B1u) >> (32 - kWalkFilterLog2);
}
__device__ __forceinline__ unsigned long long walk_filter_mask(int32_t v)
{
    const uint32_t h = (uint32_t)v * 0x85EBCA77u;
    return (1ull << (h >> 26)) | (1ull << ((h >> 20) & 63u)) | (1ull << ((h >> 14) & 63u));
}

// blocks per column of the global sparse hop 2: at least kPushSplit, up to
// kPushSplitMax when few columns take that path (hub columns)
constexpr int kPushSplit = 8;
constexpr int kPushSplitMax = 64;
constexpr double kHop2UnitBytes = 12.0;  // profiler: 4-byte index + 8-byte accumulator per pushed entry
constexpr int kHashLoadMax = 9830;  // columns with more hop-2 work use the global path

// Where the batches of a group live.  Batch k of the group holds the pairs at
// positions [p0 + k B, min(p0 + (k+1) B, pend)) of qs.ord and owns slot k:
// three n x kCols value buffers (H1, A, B) with their support bits, per-column
// statistics and mask words.  Kernels that cover a whole group take the slot
// from the grid.
struct SlotArgs {
    int64_t p0, pend;
    int32_t B;
    int32_t G;            // slots of the mask-word layout below
    char *pool;           // value buffers, slot-major
    uint32_t *bits;       // support bits, same layout with kBitWords per node
    int64_t buf_elems;    // n * kCols
    int64_t buf_words;    // n * kBitWords
    double *cs;           // per slot: m1[kCols], m2[kCols], sd[kCols] (int64)
    double *hpart;        // per slot: m1, m2, sd, each kPushSplitMax x kCols
    uint64_t *meta;       // [0,G) active masks, [G,2G) hop-2 masks, [2G,6G) hop-2 paths
};

__host__ __device__ inline int64_t slot_q0(const SlotArgs &a, int k) { return a.p0 + (int64_t)k * a.B; }
__host__ __device__ inline int slot_nb(const SlotArgs &a, int k)
{
    const int64_t r = a.pend - slot_q0(a, k);
    return (int)(r < a.B ? (r > 0 ? r : 0) : a.B);
}
__host__ __device__ inline int64_t slot_elem_off(const SlotArgs &a, int k, int which)
{
    return ((int64_t)k * 3 + which) * a.buf_elems;
}
template <class T> __host__ __device__ inline T *slot_buf(const SlotArgs &a, int k, int which)
{
    return reinterpret_cast<T *>(a.pool) + slot_elem_off(a, k, which);
}
__host__ __device__ inline uint32_t *slot_bits(const SlotArgs &a, int k, int which)
{
    return a.bits + ((int64_t)k * 3 + which) * a.buf_words;
}
__host__ __device__ inline double *slot_cs(const SlotArgs &a, int k) { return a.cs + (size_t)k * 3 * kCols; }
__host__ __device__ inline double *slot_hpart(const SlotArgs &a, int k)
{
    return a.hpart + (size_t)k * 3 * kPushSplitMax * kCols;
}

struct HopArgs {
    const void *in;          // n x kCols values (previous hop)
    void *out;               // n x kCols values (this hop)
    const uint32_t *in_bits; // n x kBitWords
    uint32_t *out_bits;
    const uint64_t *mask;    // active pairs of the batch (bit j = pair j)
    uint64_t host_mask;      // the same mask as seen by the host (for byte accounting)
    double *cs;              // column statistics of the batch's slot
    int col0, col_tile;      // column slice of this launch
};

struct QueryCtx {
    QState qs;
    int64_t nq;
    double lambda, delta;
    int32_t tau, schedule;
    uint64_t seed;
    int64_t qid_offset;
    hipStream_t stream;
    int32_t ell_rule = 0;  // 0: Eq. (ell) per pair, 1: Eq. (old-ell)
    // hop 1 from graph constants: its statistics and r_b term come from
    // per-node tables, and the hop-1 vector is scattered only for the pairs
    // that read it (walks that cannot evaluate it from LDS rows, dense hop 2)
    bool hop1_implicit = false;
};

geer_status launch_init_queries(geer_graph *g, const QueryCtx &c, const int32_t *d_fixed,
                                int32_t forced_hops, hipStream_t st);
// hop 1 (or, with clear, its reset) for slots [0, nslots)
geer_status launch_hop1_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int nslots,
                              bool clear, hipStream_t st);
// selective hop-1 scatter for slots [slot0, slot0 + nslots): kHop1Stopped
// writes the pairs stopped after hop 1 whose walks read the vector,
// kHop1Continuing the pairs that go on to a dense hop 2, kHop1Clear resets
// every pair written by either
enum { kHop1Stopped = 0, kHop1Continuing = 1, kHop1Clear = 2 };
geer_status launch_hop1_select(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int slot0,
                               int nslots, int mode, hipStream_t st);
geer_status launch_hop_dense(geer_graph *g, const HopArgs &a, int value_size, hipStream_t st);
// reserve the buffers of a dense hop (partial statistics, heavy-row segments)
geer_status reserve_dense(geer_graph *g, int value_size);
// epilogue of hop `hop` (vectors in buffer `which`) for slots [0, nslots)
geer_status launch_epilogue_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa,
                                  int nslots, int hop, int which, int value_size, hipStream_t st);
// global-path sparse hop 2, slots [slot0, slot0 + nslots): mode 0 push,
// 1 convert (+ statistics into partial rows [0, split) of the slot's hop-2
// partials), 2 clear; split blocks per column (kPushSplit..kPushSplitMax)
geer_status launch_hop2_sparse(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int slot0,
                               int nslots, int value_size, int mode, int split, hipStream_t st);
// blocks per column for a global hop-2 pass over `ncols` columns
int hop2_split(int ncols);
geer_status launch_zero(geer_graph *g, void *p, size_t bytes, hipStream_t st);
// walk filters of group positions [0, nq) from q0 (after the group's SMM)
geer_status launch_walk_filter(geer_graph *g, const QueryCtx &c, int64_t q0, int nq,
                               unsigned long long *filter, hipStream_t st);
// make at least min(want, what fits) slots of hop-2 accumulators available;
// returns the slot count (0 with *err set on failure)
int ensure_hop2_acc(geer_graph *g, int want, hipStream_t st, geer_status *err);
geer_status launch_hop2_lds_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa,
                                  int nslots, int value_size, hipStream_t st);
// hop-2 partials (rows [0, split)) -> column statistics for the pairs in each
// slot's hop-2 mask
geer_status launch_colstat_group(geer_graph *g, const SlotArgs &sa, int nslots, int split,
                                 hipStream_t st);
// largest and second-largest entry of columns [0, ncols) of a node-major
// vector buffer with `stride` values per node -> cs_m1[c], cs_m2[c]
geer_status launch_column_top2(const geer_graph *g, const void *vec, int ncols, int stride,
                               int value_size, double *cs_m1, double *cs_m2, hipStream_t st);

struct AmcGroup {
    int64_t q0;      // first query of the group
    int64_t nq;      // queries in the group
    const void *pool;
    int value_size;
    int vstride = kCols;  // values per node in the vector buffer (kCols, or 2 for one pair)
    // fixed plan (no host read; capturable): run exactly `rounds` rounds on a
    // full persistent grid with the chunk partials in the reserved zpart
    // buffer of zpart_cap entries; a round needing more sets bit 0 of
    // *sticky (a batch of 2^32 walk pairs or more: bit 1), after which no
    // round walks or updates anything
    bool fixed_plan = false;
    int rounds = 0;
    int64_t zpart_cap = 0;
    int64_t *sticky = nullptr;
    // per group position: walk filter (kWalkFilterWords words; nullptr: none)
    const unsigned long long *filter = nullptr;
};

// AMC buffers supplied by the caller instead of the workspace (nothing is
// reserved, no profiling): chunk_off[nq + 1], misc[kMiscWords], and room for
// zpart_cap chunk partials; a group needing more chunks fails with GEER_E_OOM.
struct AmcScratch {
    int64_t *chunk_off;
    int64_t *misc;
    double2 *zpart;
    int64_t zpart_cap;
};

geer_status amc_phase(geer_graph *g, const QueryCtx &c, const AmcGroup &grp, hipStream_t st,
                      int walk_ilp, const AmcScratch *ext = nullptr);
// Algorithm 1 for the single query at slot 0 of qs with caller vectors at
// element offset voff: sets s, t, ord, l_f and psi, eta*, eta_1 from the
// top-2 entries in cs_m1[0..1], cs_m2[0..1] (Eq. Delta-st, Eq. etas-star)
geer_status launch_amc_setup(const geer_graph *g, const QState &qs, int32_t s, int32_t t,
                             int32_t lf, double eps, int32_t tau, double delta, int64_t voff,
                             const double *cs_m1, const double *cs_m2, hipStream_t st);
geer_status launch_finalize(geer_graph *g, const QueryCtx &c, double *d_r_out,
                            geer_query_stats *d_stats, hipStream_t st);
geer_status launch_walk_traces(geer_graph *g, int32_t nw, const int32_t *start, const uint32_t *q,
                               const uint32_t *batch, const uint32_t *k, const uint32_t *side,
                               int32_t lf, uint64_t seed, int32_t *trace, hipStream_t st);

// Profiling helpers (graph.hip): bracket a launch with events when enabled.
int prof_begin(geer_graph *g, hipStream_t st);
void prof_end(geer_graph *g, int token, int kind, double bytes, double units, hipStream_t st);
// host-known work of a launch (and its algorithmic bytes) booked on a kind
void prof_add_units(geer_graph *g, int kind, double units, double bytes = 0.0);
// A device slot of two int64 counters for a counted record, or nullptr when
// profiling is off (kernels then write their counts to scratch).
int64_t *prof_counter(geer_graph *g, int *index);
void prof_end_counted(geer_graph *g, int token, int kind, int counter, double per_unit,
                      double per_unit2, hipStream_t st);

geer_status launch_learned(geer_graph *g, const QueryCtx &c, const geer_model *m, float *d_feat,
                           int32_t tau_max, hipStream_t st);

// every workspace buffer of a graph handle (graph.hip)
std::vector<DevBuf *> workspace_bufs(geer_graph *g);

// Workspace helpers (query.hip)
size_t qstate_bytes(int64_t cap);                      // bytes of the QState arrays for cap queries
void qstate_carve(char *base, int64_t cap, QState *qs);  // lay them out at base
geer_status ensure_qstate(geer_graph *g, int64_t nq, QState *qs);
geer_status ensure_slots(geer_graph *g, int slots, int value_size);
int grid_blocks_dense(const geer_graph *g);

}  // namespace geer
