// AMC phase (Algorithm 1 as called from Algorithm 3): adaptive batches of
// walk pairs from the SMM frontier, stopped by the empirical-Bernstein rule.
//
// Work decomposition: in batch i a query needs eta_i = eta_1 * 2^i walk
// pairs.  Pairs are cut into chunks of 32; a wavefront takes one chunk
// (lanes 2k and 2k+1 walk S_k from s and T_k from t).  Chunk offsets come
// from a prefix sum over the group's queries, so a persistent grid can
// stride over all chunks of all queries of a group in one launch.  Each chunk
// writes (sum Z, sum Z^2) to its own slot and the stop kernel adds the slots
// of a query in a fixed order: results do not depend on scheduling.
//
// A walk step costs one random line fill for its walk record.  The pair's
// vector values at the new node come from LDS rows (one-hop vectors of short
// rows), from the node itself (indicator vectors), or from the batch slots,
// read only when the pair's support filter admits the node (off the supports
// the values are exact zeros).  Each step requests the next step's record
// before it consumes its own values, so the two are in flight together.
#include <type_traits>

#include "geer_internal.h"

namespace geer {

template <class T> struct Val2;
template <> struct Val2<float> { using type = float2; };
template <> struct Val2<double> { using type = double2; };

constexpr int kWalkBlocksPerCu = 7;
// Each round's chunks are walked by two launches (each a contiguous half,
// split over the XCDs).  The other stream's kernels start mostly while a walk
// launch drains, so a second drain point per round lets the next group's SMM
// advance; on the 1M-node Chung-Lu workload 1, 2, 3 and 4 parts gave 219-221K,
// 221.8-222.8K, 220.8K and 219.3K pairs/s.
constexpr int kWalkParts = 2;

__device__ __forceinline__ bool one_hop_from_graph(int32_t lb, int32_t ds, int32_t dt)
{
    return lb == 1 && ds <= kMemberRowMax && dt <= kMemberRowMax;
}

// ----------------------------------------------------------------------------
// plan: chunk prefix sums for batch `round` of the active queries of a group
// ----------------------------------------------------------------------------

// sticky (nullable): a fixed plan's overflow word.  Once it is set no chunk
// is planned; a round whose chunks exceed cap sets it (bit 0) and plans none.
__global__ __launch_bounds__(1024) void k_amc_plan(QState qs, int64_t q0, int nq, int round,
                                                   int64_t *__restrict__ chunk_off,
                                                   int64_t *__restrict__ total,
                                                   int64_t *__restrict__ steps,
                                                   const int32_t *__restrict__ row_ptr,
                                                   int64_t cap, int64_t *__restrict__ sticky)
{
    __shared__ int64_t s_sum[1024];
    __shared__ unsigned long long s_steps, s_vsteps;
    if (threadIdx.x == 0) s_steps = s_vsteps = 0;
    __syncthreads();
    const bool halt = sticky && *sticky != 0;
    const int tid = threadIdx.x;
    const int per = (nq + 1023) / 1024;
    const int a = min(nq, tid * per), b = min(nq, a + per);
    int64_t local = 0;
    for (int i = a; i < b; ++i) {
        int64_t q = qs.ord[q0 + i];
        if (!halt && qs.active_amc[q]) {
            int64_t eta = qs.eta1[q] << round;
            local += (eta + kPairsPerChunk - 1) / kPairsPerChunk;
            const unsigned long long st = (unsigned long long)(2 * eta * qs.lf[q]);
            atomicAdd(&s_steps, st);
            const int32_t s = qs.s[q], t = qs.t[q];
            if (qs.vec_off[q] >= 0 &&
                !one_hop_from_graph(qs.lb[q], row_ptr[s + 1] - row_ptr[s], row_ptr[t + 1] - row_ptr[t]))
                atomicAdd(&s_vsteps, st);
        }
    }
    s_sum[tid] = local;
    __syncthreads();
    // inclusive Hillis-Steele scan over the 1024 per-thread sums
    for (int o = 1; o < 1024; o <<= 1) {
        int64_t v = tid >= o ? s_sum[tid - o] : 0;
        __syncthreads();
        s_sum[tid] += v;
        __syncthreads();
    }
    int64_t run = s_sum[tid] - local;  // exclusive prefix of this thread's range
    for (int i = a; i < b; ++i) {
        chunk_off[i] = run;
        int64_t q = qs.ord[q0 + i];
        if (!halt && qs.active_amc[q]) {
            int64_t eta = qs.eta1[q] << round;
            run += (eta + kPairsPerChunk - 1) / kPairsPerChunk;
        }
    }
    if (tid == 1023) {
        chunk_off[nq] = s_sum[1023];
        *total = s_sum[1023];
        if (sticky && s_sum[1023] > cap) {
            *sticky |= 1;
            *total = 0;
        }
        steps[0] = (int64_t)s_steps;
        steps[1] = (int64_t)s_vsteps;
    }
}

// Upper bound of the chunks of any batch of a group: every pair's largest
// batch is its last (eta_1 2^(tau_q - 1)), so the sum of those chunk counts
// bounds every round's total.  out: [0] the bound, [1] overflow flag (a batch
// of 2^32 walk pairs or more), [2] the largest per-pair batch count.
// With a fixed plan, sticky (nullable) records a too large batch (bit 1)
// for the whole call.
__global__ __launch_bounds__(1024) void k_amc_bound(QState qs, int64_t q0, int nq,
                                                    int64_t *__restrict__ out,
                                                    int64_t *__restrict__ sticky)
{
    __shared__ unsigned long long s_chunks;
    __shared__ int s_over, s_tau;
    if (threadIdx.x == 0) {
        s_chunks = 0;
        s_over = 0;
        s_tau = 0;
    }
    __syncthreads();
    unsigned long long chunks = 0;
    int over = 0, tmax = 0;
    for (int i = threadIdx.x; i < nq; i += blockDim.x) {
        const int64_t q = qs.ord[q0 + i];
        if (!qs.active_amc[q]) continue;
        const int tq = qs.tau_q[q];
        const int64_t e1 = qs.eta1[q];
        // eta_1 2^(tq - 1) >= 2^32  <=>  eta_1 >= 2^(33 - tq)
        if (tq > 33 || e1 >= (int64_t(1) << (33 - tq))) {
            over = 1;
            continue;
        }
        const int64_t eta = e1 << (tq - 1);
        chunks += (unsigned long long)((eta + kPairsPerChunk - 1) / kPairsPerChunk);
        tmax = max(tmax, tq);
    }
    atomicAdd(&s_chunks, chunks);
    if (over) atomicOr(&s_over, 1);
    atomicMax(&s_tau, tmax);
    __syncthreads();
    if (threadIdx.x == 0) {
        out[0] = (int64_t)s_chunks;
        out[1] = s_over;
        out[2] = s_tau;
        if (sticky && s_over) *sticky |= 2;
    }
}

// ----------------------------------------------------------------------------
// walks
// ----------------------------------------------------------------------------

// Walk records (one per CSR entry, see geer_graph::d_walk_rec): 8-byte
// packed {v | b << sb | d << sd} when the bit widths of n, nnz and the largest
// degree fit 64 bits, else 16-byte {v, b, d, -}.
template <int RB> struct WalkRec;
template <> struct WalkRec<8> {
    using Raw = uint64_t;
    static __device__ __forceinline__ Raw fetch(const void *rec, int64_t e)
    {
        return __builtin_nontemporal_load(static_cast<const uint64_t *>(rec) + e);
    }
    static __device__ __forceinline__ void decode(Raw x, uint32_t sb, uint32_t sd, int32_t &v, int32_t &b,
                                                  int32_t &d)
    {
        v = (int32_t)(x & ((1ull << sb) - 1));
        b = (int32_t)((x >> sb) & ((1ull << (sd - sb)) - 1));
        d = (int32_t)(x >> sd);
    }
};
template <> struct WalkRec<16> {
    using Raw = int4;
    static __device__ __forceinline__ Raw fetch(const void *rec, int64_t e)
    {
        return static_cast<const int4 *>(rec)[e];
    }
    static __device__ __forceinline__ void decode(Raw x, uint32_t, uint32_t, int32_t &v, int32_t &b, int32_t &d)
    {
        v = x.x;
        b = x.y;
        d = x.z;
    }
};

// x in the sorted row held in LDS (kMemberRowMax entries, padded with INT32_MAX)
__device__ __forceinline__ bool lds_row_contains(const int32_t *row, int32_t x)
{
    int pos = 0;
#pragma unroll
    for (int step = kMemberRowMax / 2; step > 0; step >>= 1)
        if (row[pos + step - 1] < x) pos += step;
    return row[pos] == x;
}

// Groups up to this many pairs keep their chunk offsets in LDS.
constexpr int kChunkOffLds = 2048;
constexpr int kXcds = 8;  // accelerator complex dies of an MI355X

// VS: values per node in the vector buffer (kCols for batch slots, 2 for one
// pair's caller vectors)
template <class T, int RB, int VS>
__global__ __launch_bounds__(256) void k_walk(QState qs, int64_t q0, int nq, int round,
                                              const int64_t *__restrict__ chunk_off,
                                              const int64_t *__restrict__ total_p,
                                              const int32_t *__restrict__ row_ptr,
                                              const int32_t *__restrict__ col_idx,
                                              const void *__restrict__ rec, uint32_t rec_sb,
                                              uint32_t rec_sd, const T *__restrict__ pool,
                                              uint32_t key0, uint32_t key1, int64_t qid_offset,
                                              double2 *__restrict__ zpart, int part, int nparts,
                                              const unsigned long long *__restrict__ filter)
{
    using T2 = typename Val2<T>::type;
    // chunk offsets in LDS as 32-bit values when they fit
    __shared__ int32_t s_off[kChunkOffLds + 1];
    // per wave: the sorted rows of s and t of its current chunk's pair
    __shared__ int32_t s_rows[4][2][kMemberRowMax];
    const int64_t total = *total_p;
    const bool lds_off = nq <= kChunkOffLds && total < (int64_t(1) << 31);
    if (lds_off)
        for (int i = threadIdx.x; i <= nq; i += blockDim.x) s_off[i] = (int32_t)chunk_off[i];
    __syncthreads();
    auto off = [&](int i) -> int64_t { return lds_off ? (int64_t)s_off[i] : chunk_off[i]; };
    const int lane = threadIdx.x & 63;
    const int wv = threadIdx.x >> 6;
    // Blocks are dealt to the 8 XCDs round-robin; XCD x takes the x-th eighth
    // of the chunks (chunks are ordered by batch slot), so the vector rows its
    // walks revisit belong to few slots and can stay in that XCD's L2.
    const int nx = gridDim.x % kXcds == 0 ? kXcds : 1;
    const int xcd = blockIdx.x % nx;
    // this launch's part of the round's chunks, then the XCD's share of it
    const int64_t p_lo = total * part / nparts, span = total * (part + 1) / nparts - p_lo;
    const int64_t c_lo = p_lo + span * xcd / nx, c_hi = p_lo + span * (xcd + 1) / nx;
    const int64_t gw = (int64_t)(blockIdx.x / nx) * 4 + wv;
    const int64_t nw = (int64_t)(gridDim.x / nx) * 4;
    const uint32_t side = lane & 1;
    for (int64_t c = c_lo + gw; c < c_hi; c += nw) {
        // pair of this chunk: largest i with off[i] <= c
        int lo = 0, hi = nq;
        while (hi - lo > 1) {
            int mid = (lo + hi) >> 1;
            if (off(mid) <= c) lo = mid;
            else hi = mid;
        }
        const int64_t q = qs.ord[q0 + lo];
        const int64_t eta = qs.eta1[q] << round;
        const int64_t k = (c - off(lo)) * kPairsPerChunk + (lane >> 1);
        const bool valid = k < eta;
        const int32_t s = qs.s[q], t = qs.t[q];
        const int32_t lf = qs.lf[q];
        const int64_t voff = qs.vec_off[q];
        const int32_t bs = row_ptr[s], ds = row_ptr[s + 1] - bs;
        const int32_t bt = row_ptr[t], dt = row_ptr[t + 1] - bt;
        const double ids = 1.0 / ds, idt = 1.0 / dt;
        // one-hop vectors: s*(u) = 1/d(u) on N(s), t*(u) = 1/d(u) on N(t)
        // (the values the hop-1 scatter stored), evaluated from the graph
        const bool member = voff >= 0 && one_hop_from_graph(qs.lb[q], ds, dt);
        // pairs with a walk filter read their values only at nodes it holds
        const unsigned long long *fq =
            filter && walk_filtered(voff, qs.lb[q], ds, dt) ? filter + (size_t)lo * kWalkFilterWords : nullptr;
        if (member) {
            // the wave's previous reads of s_rows have completed (their values
            // were consumed), so the rows can be overwritten in place
            for (int i = lane; i < kMemberRowMax; i += 64) {
                s_rows[wv][0][i] = i < ds ? col_idx[bs + i] : INT32_MAX;
                s_rows[wv][1][i] = i < dt ? col_idx[bt + i] : INT32_MAX;
            }
            __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
            __builtin_amdgcn_wave_barrier();
            __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
        }
        const uint32_t qid = (uint32_t)(q + qid_offset);
        const uint32_t c2 = ((uint32_t)round << 1) | side;
        double acc = 0.0;
        if (valid && lf > 0) {
            int32_t b = side ? bt : bs, d = side ? dt : ds;
            uint4 r4 = philox4x32_10(make_uint4(0u, (uint32_t)k, c2, qid), key0, key1);
            // One loop per kind of pair (wave-uniform), so that no load sits
            // behind a branch.  The node after a step is row u's (draw mod
            // d(u))-th entry; its record also carries that node's row start and
            // degree.  The record of step + 1 is requested after this step's
            // filter word or values and before they are used: loads complete
            // in order, so they can be consumed while the record is in flight.
            // kind 0: indicator vectors, 1: one-hop vectors from LDS rows,
            // 2: slot values behind a walk filter, 3: slot values.
            auto walk = [&](auto kind) {
                constexpr int K = decltype(kind)::value;
                auto early = [&](int32_t u, unsigned long long &fw, T2 &pv) {
                    if constexpr (K == 2) fw = fq[walk_filter_word(u)];
                    if constexpr (K == 3) pv = *reinterpret_cast<const T2 *>(pool + voff + (size_t)u * VS);
                };
                auto add = [&](int32_t u, int32_t du, unsigned long long fw, T2 pv) {
                    double xv, yv;
                    if constexpr (K == 0) {
                        xv = u == s ? 1.0 : 0.0;
                        yv = u == t ? 1.0 : 0.0;
                    } else if constexpr (K == 1) {
                        const double inv = (double)(T)(1.0 / (double)du);
                        xv = lds_row_contains(s_rows[wv][0], u) ? inv : 0.0;
                        yv = lds_row_contains(s_rows[wv][1], u) ? inv : 0.0;
                    } else if constexpr (K == 2) {
                        if ((fw & walk_filter_mask(u)) != walk_filter_mask(u)) {
                            xv = 0.0;  // u is in neither support
                            yv = 0.0;
                        } else {
                            const T2 w = *reinterpret_cast<const T2 *>(pool + voff + (size_t)u * VS);
                            xv = (double)w.x;
                            yv = (double)w.y;
                        }
                    } else {
                        xv = (double)pv.x;
                        yv = (double)pv.y;
                    }
                    // Z_k: S_k adds s(u)/d(s) - t(u)/d(t); T_k adds t(u)/d(t) - s(u)/d(s)
                    acc += side ? (yv * idt - xv * ids) : (xv * ids - yv * idt);
                };
                typename WalkRec<RB>::Raw raw =
                    WalkRec<RB>::fetch(rec, b + (int32_t)(pick_word(r4, 0u) % (uint32_t)d));
                int32_t u;
                for (int32_t step = 0; step + 1 < lf; ++step) {
                    WalkRec<RB>::decode(raw, rec_sb, rec_sd, u, b, d);
                    unsigned long long fw = 0ull;
                    T2 pv{};
                    early(u, fw, pv);
                    __builtin_amdgcn_sched_barrier(0);
                    const uint32_t ns = (uint32_t)step + 1u;
                    if ((ns & 3u) == 0)
                        r4 = philox4x32_10(make_uint4(ns >> 2, (uint32_t)k, c2, qid), key0, key1);
                    raw = WalkRec<RB>::fetch(rec, b + (int32_t)(pick_word(r4, ns & 3u) % (uint32_t)d));
                    __builtin_amdgcn_sched_barrier(0);
                    add(u, d, fw, pv);
                }
                WalkRec<RB>::decode(raw, rec_sb, rec_sd, u, b, d);
                unsigned long long fw = 0ull;
                T2 pv{};
                early(u, fw, pv);
                add(u, d, fw, pv);
            };
            if (voff < 0) walk(std::integral_constant<int, 0>{});
            else if (member) walk(std::integral_constant<int, 1>{});
            else if (fq) walk(std::integral_constant<int, 2>{});
            else walk(std::integral_constant<int, 3>{});
        }
        const double z = acc + __shfl_xor(acc, 1);
        double zs = (valid && side == 0) ? z : 0.0;
        double z2 = zs * zs;
#pragma unroll
        for (int o = 1; o < 64; o <<= 1) {
            zs += __shfl_xor(zs, o);
            z2 += __shfl_xor(z2, o);
        }
        if (lane == 0) zpart[c] = make_double2(zs, z2);
    }
}

// ----------------------------------------------------------------------------
// walk filters (one block per group position)
// ----------------------------------------------------------------------------

// Inserts supp(x) U supp(y) of each filtered pair that still walks: N(s) and
// N(t) at depth 1, the nodes two hops from s or t at depth 2 (every node a
// hop-2 vector can be nonzero on).  Built in LDS, then written out whole.
__global__ __launch_bounds__(256) void k_walk_filter(QState qs, int64_t q0, const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col_idx,
                                                     unsigned long long *__restrict__ filter)
{
    __shared__ unsigned long long f[kWalkFilterWords];
    const int64_t q = qs.ord[q0 + blockIdx.x];
    const int32_t s = qs.s[q], t = qs.t[q], lb = qs.lb[q];
    const int32_t bs = row_ptr[s], ds = row_ptr[s + 1] - bs;
    const int32_t bt = row_ptr[t], dt = row_ptr[t + 1] - bt;
    if (!qs.active_amc[q] || !walk_filtered(qs.vec_off[q], lb, ds, dt)) return;
    for (int w = threadIdx.x; w < kWalkFilterWords; w += blockDim.x) f[w] = 0ull;
    __syncthreads();
    auto insert = [&](int32_t v) { atomicOr(&f[walk_filter_word(v)], walk_filter_mask(v)); };
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6, waves = blockDim.x >> 6;
    for (int side = 0; side < 2; ++side) {
        const int32_t b = side ? bt : bs, d = side ? dt : ds;
        if (lb == 1) {
            for (int k = threadIdx.x; k < d; k += blockDim.x) insert(col_idx[b + k]);
        } else {
            for (int k = wave; k < d; k += waves) {
                const int32_t v = col_idx[b + k];
                const int32_t bv = row_ptr[v], dv = row_ptr[v + 1] - bv;
                for (int m = lane; m < dv; m += 64) insert(col_idx[bv + m]);
            }
        }
    }
    __syncthreads();
    unsigned long long *out = filter + (size_t)blockIdx.x * kWalkFilterWords;
    for (int w = threadIdx.x; w < kWalkFilterWords; w += blockDim.x) out[w] = f[w];
}

geer_status launch_walk_filter(geer_graph *g, const QueryCtx &c, int64_t q0, int nq, unsigned long long *filter,
                               hipStream_t st)
{
    if (nq <= 0) return GEER_OK;
    hipLaunchKernelGGL(k_walk_filter, dim3(nq), dim3(256), 0, st, c.qs, q0, g->d_row_ptr, g->d_col_idx, filter);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// stop rule after batch `round` (one wavefront per query)
// ----------------------------------------------------------------------------

__global__ __launch_bounds__(256) void k_amc_stop(QState qs, int64_t q0, int nq, int round,
                                                  const int64_t *__restrict__ chunk_off,
                                                  const double2 *__restrict__ zpart, int32_t tau,
                                                  double delta, const int64_t *__restrict__ sticky)
{
    if (sticky && *sticky) return;  // a fixed plan overflowed: the call fails
    const int lane = threadIdx.x & 63;
    const int i = blockIdx.x * 4 + (threadIdx.x >> 6);
    if (i >= nq) return;
    const int64_t q = qs.ord[q0 + i];
    if (!qs.active_amc[q]) return;
    double zs = 0.0, z2 = 0.0;
    for (int64_t c = chunk_off[i] + lane; c < chunk_off[i + 1]; c += 64) {
        double2 p = zpart[c];
        zs += p.x;
        z2 += p.y;
    }
#pragma unroll
    for (int o = 1; o < 64; o <<= 1) {
        zs += __shfl_xor(zs, o);
        z2 += __shfl_xor(z2, o);
    }
    if (lane != 0) return;
    const double eta = (double)(qs.eta1[q] << round);
    const double z = zs / eta;
    double var = z2 / eta - z * z;
    if (var < 0.0) var = 0.0;
    tau = qs.tau_q[q];
    const double f = bernstein_of(eta, var, qs.psi[q], delta / (double)tau);
    qs.batches[q] = round + 1;
    qs.walk_pairs[q] += qs.eta1[q] << round;
    qs.zsum[q] = zs;
    qs.z2sum[q] = z2;
    qs.var[q] = var;
    qs.f[q] = f;
    qs.rf[q] = z;
    if (f <= qs.eps[q] / 2.0) {
        qs.active_amc[q] = 0;
        qs.stop[q] = GEER_STOP_BERNSTEIN;
    } else if (round + 1 >= tau) {
        qs.active_amc[q] = 0;
        qs.stop[q] = GEER_STOP_CAP;
    }
}

geer_status amc_phase(geer_graph *g, const QueryCtx &c, const AmcGroup &grp, hipStream_t st,
                      int walk_ilp, const AmcScratch *ext)
{
    (void)walk_ilp;
    Workspace &ws = g->ws;
    if (grp.nq <= 0) return GEER_OK;
    if (grp.vstride != kCols && grp.vstride != 2)
        return fail(GEER_E_INVALID_ARG, "vector stride must be 128 or 2");
    const int nq = (int)grp.nq;
    if (!ext) GEER_TRY(ws.chunk_off.reserve(((size_t)nq + 1) * sizeof(int64_t)));
    int64_t *chunk_off = ext ? ext->chunk_off : ws.chunk_off.as<int64_t>();
    int64_t *misc = ext ? ext->misc : ws.misc.as<int64_t>();
    int64_t *d_total = misc + 8;
    int64_t *d_bound = misc + 12;
    // The chunk bound sizes the partials and the grid.  Normally it is read
    // once per group and the rounds then run without host synchronisation
    // (rounds in which no pair is left launch empty grids).  A fixed plan
    // reads nothing: it runs its given rounds on a full grid over the
    // reserved partials, and a round that would not fit sets the overflow word.
    int64_t *sticky = grp.fixed_plan ? grp.sticky : nullptr;
    hipLaunchKernelGGL(k_amc_bound, dim3(1), dim3(1024), 0, st, c.qs, grp.q0, nq, d_bound, sticky);
    GEER_HIP(hipGetLastError());
    int64_t bound = 0;
    int rounds = 0;
    if (grp.fixed_plan) {
        if (ext || !grp.sticky) return fail(GEER_E_INVALID_ARG, "fixed AMC plan needs the workspace partials");
        bound = grp.zpart_cap;
        rounds = std::min(grp.rounds, (int)c.tau);
        if ((size_t)bound * sizeof(double2) > ws.zpart.bytes)
            return fail(GEER_E_DEVICE, "fixed AMC plan: partials not reserved");
    } else {
        int64_t host[3] = {0, 0, 0};
        GEER_HIP(hipMemcpyAsync(host, d_bound, 3 * sizeof(int64_t), hipMemcpyDeviceToHost, st));
        GEER_HIP(hipStreamSynchronize(st));
        if (host[1] != 0) return fail(GEER_E_INVALID_ARG, "AMC batch exceeds 2^32 walk pairs for a query");
        bound = host[0];
        rounds = (int)std::min<int64_t>(host[2], c.tau);
        if (ext) {
            if (bound > ext->zpart_cap)
                return fail(GEER_E_OOM, "scratch cap exceeded: the AMC batches need " + std::to_string(bound) +
                                            " chunk partials, the fixed scratch holds " +
                                            std::to_string(ext->zpart_cap));
        } else if (bound > 0) {
            GEER_TRY(ws.zpart.reserve((size_t)bound * sizeof(double2)));
        }
    }
    if (bound == 0 || rounds <= 0) return GEER_OK;
    // a CU holds 8 walk workgroups (32 VGPRs, 17 KB of LDS, 4 waves each);
    // the grid fills 7 of them, so the next group's SMM kernels, queued on the
    // other stream, always find room beside the walks.  (Results do not depend
    // on the grid: a chunk's partial is the same whichever wave walks it.)
    int blocks = (int)std::min<int64_t>((bound + 3) / 4, (int64_t)g->num_cus * kWalkBlocksPerCu);
    if (blocks >= kXcds) blocks -= blocks % kXcds;  // whole rounds over the XCDs
    const uint32_t key0 = (uint32_t)c.seed, key1 = (uint32_t)(c.seed >> 32);
    const void *rec = g->d_walk_rec;
    const uint32_t sb = (uint32_t)g->rec_sb, sd = (uint32_t)g->rec_sd;
    auto *zp = ext ? ext->zpart : ws.zpart.as<double2>();
    const unsigned long long *filt = grp.vstride == kCols ? grp.filter : nullptr;
    for (int round = 0; round < rounds; ++round) {
        // walk steps of the batch (all, and those reading SMM vectors) for the
        // profiler's byte count, else into scratch
        int counter = -1;
        int64_t *d_steps = ext ? nullptr : prof_counter(g, &counter);
        if (!d_steps) d_steps = misc + 10;
        hipLaunchKernelGGL(k_amc_plan, dim3(1), dim3(1024), 0, st, c.qs, grp.q0, nq, round,
                           chunk_off, d_total, d_steps, g->d_row_ptr, grp.zpart_cap, sticky);
        GEER_HIP(hipGetLastError());
        for (int part = 0; part < kWalkParts; ++part) {
            int tok = ext ? -1 : prof_begin(g, st);
#define GEER_WALK_LAUNCH(T, RB, VS)                                                                 \
    hipLaunchKernelGGL((k_walk<T, RB, VS>), dim3(blocks), dim3(256), 0, st, c.qs, grp.q0, nq, round, \
                       chunk_off, d_total, g->d_row_ptr, g->d_col_idx, rec, sb, sd,                 \
                       (const T *)grp.pool, key0, key1, c.qid_offset, zp, part, kWalkParts, filt)
#define GEER_WALK_LAUNCH_T(T, VS)                       \
    do {                                                \
        if (g->walk_rec_bytes == 8) GEER_WALK_LAUNCH(T, 8, VS); \
        else GEER_WALK_LAUNCH(T, 16, VS);               \
    } while (0)
            if (grp.vstride == kCols) {
                if (grp.value_size == 4) GEER_WALK_LAUNCH_T(float, kCols);
                else GEER_WALK_LAUNCH_T(double, kCols);
            } else {
                if (grp.value_size == 4) GEER_WALK_LAUNCH_T(float, 2);
                else GEER_WALK_LAUNCH_T(double, 2);
            }
#undef GEER_WALK_LAUNCH_T
#undef GEER_WALK_LAUNCH
            GEER_HIP(hipGetLastError());
            // per step: one walk record; steps of pairs whose vectors are
            // read also fetch the pair's two values at the new node (the
            // round's steps are booked on its last launch)
            if (part + 1 < kWalkParts) prof_end(g, tok, PK_WALK, 0.0, 0.0, st);
            else prof_end_counted(g, tok, PK_WALK, counter, (double)g->walk_rec_bytes,
                                  2.0 * grp.value_size, st);
        }
        hipLaunchKernelGGL(k_amc_stop, dim3((nq + 3) / 4), dim3(256), 0, st, c.qs, grp.q0, nq,
                           round, chunk_off, zp, c.tau, c.delta, sticky);
        GEER_HIP(hipGetLastError());
    }
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// one pair on caller vectors (Algorithm 1 as a phase of its own)
// ----------------------------------------------------------------------------

__global__ void k_amc_setup(QState qs, const int32_t *__restrict__ row_ptr, int32_t s, int32_t t,
                            int32_t lf, double eps, int32_t tau, double delta, int64_t voff,
                            const double *__restrict__ cs_m1, const double *__restrict__ cs_m2)
{
    const double ids = 1.0 / (row_ptr[s + 1] - row_ptr[s]);
    const double idt = 1.0 / (row_ptr[t + 1] - row_ptr[t]);
    qs.s[0] = s;
    qs.t[0] = t;
    qs.ord[0] = 0;
    qs.eps[0] = eps;
    qs.ell[0] = -1;
    qs.lb[0] = -1;
    qs.lf[0] = lf;
    qs.vec_off[0] = voff;
    qs.batches[0] = 0;
    qs.walk_pairs[0] = 0;
    qs.rb[0] = 0.0;
    qs.rf[0] = 0.0;
    qs.zsum[0] = qs.z2sum[0] = qs.var[0] = qs.f[0] = 0.0;
    qs.supp_sum[0] = 0;
    qs.fallback[0] = 0;
    qs.tau_q[0] = tau;
    double psi = lf > 0 ? psi_of(lf, cs_m1[0], cs_m2[0], cs_m1[1], cs_m2[1], ids, idt) : 0.0;
    double es = lf > 0 ? eta_star_of(psi, eps, tau, delta) : 0.0;
    qs.psi[0] = psi;
    qs.eta_star[0] = es;
    qs.eta1[0] = lf > 0 ? eta1_of(es, tau) : 0;
    qs.active_amc[0] = qs.eta1[0] > 0 ? 1 : 0;
    qs.stop[0] = qs.active_amc[0] ? GEER_STOP_CAP : GEER_STOP_NO_WALKS;
}

geer_status launch_amc_setup(const geer_graph *g, const QState &qs, int32_t s, int32_t t,
                             int32_t lf, double eps, int32_t tau, double delta, int64_t voff,
                             const double *cs_m1, const double *cs_m2, hipStream_t st)
{
    hipLaunchKernelGGL(k_amc_setup, dim3(1), dim3(1), 0, st, qs, g->d_row_ptr, s, t, lf, eps, tau,
                       delta, voff, cs_m1, cs_m2);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// combine r' = r_b + r_f and write the per-query records
// ----------------------------------------------------------------------------

__global__ void k_finalize(QState qs, int64_t nq, double *__restrict__ r_out,
                           geer_query_stats *__restrict__ stats)
{
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    double r;
    if (qs.stop[q] < 0) r = __builtin_nan("");
    else if (qs.stop[q] == GEER_STOP_SAME_NODE) r = 0.0;
    else r = qs.rb[q] + qs.rf[q];
    qs.r[q] = r;
    r_out[q] = r;
    if (stats) {
        geer_query_stats st;
        st.ell = qs.ell[q];
        st.ell_b = qs.lb[q];
        st.tau = qs.tau_q[q];
        st.batches_run = qs.batches[q];
        st.stop_reason = qs.stop[q];
        st.fallback = qs.fallback[q];
        st.eta1 = qs.eta1[q];
        st.walk_pairs = qs.walk_pairs[q];
        st.supp_sum = qs.supp_sum[q];
        st.r_b = qs.stop[q] == GEER_STOP_SAME_NODE ? 0.0 : qs.rb[q];
        st.r_f = qs.rf[q];
        st.psi = qs.psi[q];
        st.eta_star = qs.eta_star[q];
        st.sigma2 = qs.var[q];
        st.f_last = qs.f[q];
        stats[q] = st;
    }
}

geer_status launch_finalize(geer_graph *g, const QueryCtx &c, double *d_r_out,
                            geer_query_stats *d_stats, hipStream_t st)
{
    (void)g;
    if (c.nq == 0) return GEER_OK;
    hipLaunchKernelGGL(k_finalize, dim3((int)((c.nq + 255) / 256)), dim3(256), 0, st, c.qs, c.nq,
                       d_r_out, d_stats);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// walk traces (same sampler as k_walk)
// ----------------------------------------------------------------------------

__global__ void k_walk_traces(int32_t nw, const int32_t *__restrict__ start,
                              const uint32_t *__restrict__ qv, const uint32_t *__restrict__ bv,
                              const uint32_t *__restrict__ kv, const uint32_t *__restrict__ sv,
                              int32_t lf, uint32_t key0, uint32_t key1,
                              const int32_t *__restrict__ row_ptr,
                              const int32_t *__restrict__ col_idx, int32_t *__restrict__ trace)
{
    int i = blockIdx.x * blockDim.x + threadIdx.x;
    if (i >= nw) return;
    int32_t u = start[i];
    const uint32_t c1 = kv[i], c2 = (bv[i] << 1) | sv[i], c3 = qv[i];
    uint4 r4 = make_uint4(0, 0, 0, 0);
    for (int32_t step = 0; step < lf; ++step) {
        if ((step & 3) == 0) r4 = philox4x32_10(make_uint4((uint32_t)step >> 2, c1, c2, c3), key0, key1);
        u = walk_next(row_ptr, col_idx, u, pick_word(r4, (uint32_t)step & 3u));
        trace[(size_t)i * lf + step] = u;
    }
}

geer_status launch_walk_traces(geer_graph *g, int32_t nw, const int32_t *start, const uint32_t *q,
                               const uint32_t *batch, const uint32_t *k, const uint32_t *side,
                               int32_t lf, uint64_t seed, int32_t *trace, hipStream_t st)
{
    hipLaunchKernelGGL(k_walk_traces, dim3((nw + 255) / 256), dim3(256), 0, st, nw, start, q,
                       batch, k, side, lf, (uint32_t)seed, (uint32_t)(seed >> 32), g->d_row_ptr,
                       g->d_col_idx, trace);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

}  // namespace geer
