// SMM phase (Algorithm 2 inside Algorithm 3): repeated products with the
// transition matrix P = D^-1 A for a batch of up to 64 pairs at once.
//
// Vectors of a batch live in an n x 128 row-major buffer: column 2j is s*_j,
// column 2j+1 is t*_j, so one pair's two values at a node are adjacent (the
// walk kernel later reads them with one 8-byte load).
//
//   hop 1:  exact sparse scatter.  (P e_u)(v) = 1/d(v) for v in N(u), 0 else.
//   hop>=2: dense pull SpMM  y(v) = (1/d(v)) sum_{u in N(v)} x(u)  over a
//           column tile.  A wavefront owns a row (degree <= 256) or a
//           256-entry segment of a heavy row; lanes own column pairs; the
//           neighbour rows are gathered with 8/16-byte loads.  Heavy-row
//           segments are summed in a second pass in fixed order, so every
//           result is deterministic (no floating-point atomics).
//   Fused into the same pass: the structural support bitmask (OR over
//   neighbours), per-column largest/second-largest value and the degree sum
//   over the support, reduced per block and then per column.
#include "geer_internal.h"

namespace geer {

template <class T> struct Vec2;
template <> struct Vec2<float> { using type = float2; };
template <> struct Vec2<double> { using type = double2; };

// Largest / second-largest with repeats counted (the second largest of
// {3, 3} is 3), branch-free: the smaller of (m1, v) competes for second place.
template <class T> __device__ __forceinline__ void top2_push(T &m1, T &m2, T v)
{
    const T lo = v < m1 ? v : m1;
    m1 = v > m1 ? v : m1;
    m2 = lo > m2 ? lo : m2;
}

// ----------------------------------------------------------------------------
// init: per-query l (Eq. ell), r_b at hop 0, schedule targets
// ----------------------------------------------------------------------------

__global__ void k_init_queries(QState qs, int64_t nq, const int32_t *__restrict__ row_ptr,
                               int32_t n, double lambda, double delta, int32_t tau,
                               int32_t schedule, const int32_t *__restrict__ fixed,
                               int32_t forced_hops, int32_t ell_rule)
{
    int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
    if (q >= nq) return;
    int32_t s = qs.s[q], t = qs.t[q];
    double eps = qs.eps[q];
    qs.batches[q] = 0;
    qs.walk_pairs[q] = 0;
    qs.eta1[q] = 0;
    qs.psi[q] = 0.0;
    qs.eta_star[q] = 0.0;
    qs.zsum[q] = qs.z2sum[q] = qs.var[q] = qs.f[q] = qs.rf[q] = 0.0;
    qs.fallback[q] = 0;
    qs.tau_q[q] = tau;
    qs.vec_off[q] = -1;
    qs.lb[q] = 0;
    qs.h1w[q] = 0;
    bool bad = s < 0 || s >= n || t < 0 || t >= n || !(eps > 0.0) || isinf(eps);
    if (bad) {
        qs.ell[q] = 0;
        qs.lf[q] = 0;
        qs.lb_target[q] = 0;
        qs.rb[q] = 0.0;
        qs.supp_sum[q] = 0;
        qs.active_smm[q] = 0;
        qs.active_amc[q] = 0;
        qs.stop[q] = -1;
        qs.r[q] = __builtin_nan("");
        return;
    }
    if (s == t && forced_hops < 0) {  // r(s,s) = 0 (Section 2.2)
        qs.ell[q] = 0;
        qs.lf[q] = 0;
        qs.lb_target[q] = 0;
        qs.rb[q] = 0.0;
        qs.supp_sum[q] = 0;
        qs.active_smm[q] = 0;
        qs.active_amc[q] = 0;
        qs.stop[q] = GEER_STOP_SAME_NODE;
        qs.r[q] = 0.0;
        return;
    }
    int32_t ds = row_ptr[s + 1] - row_ptr[s], dt = row_ptr[t + 1] - row_ptr[t];
    double ids = 1.0 / ds, idt = 1.0 / dt;
    int32_t ell = forced_hops >= 0 ? forced_hops
                  : ell_rule == 1   ? ell_peng_of(eps, lambda)
                                    : ell_of(ds, dt, eps, lambda);
    int32_t target = ell;
    if (forced_hops < 0 && schedule == GEER_SCHEDULE_FIXED)
        target = min(max(fixed[q], 0), ell);
    qs.ell[q] = ell;
    qs.lb_target[q] = target;
    qs.rb[q] = ids + idt;  // hop-0 term: e_s(s)/d(s) + e_t(t)/d(t), cross terms 0 for s != t
    qs.supp_sum[q] = (int64_t)ds + dt;
    qs.r[q] = 0.0;
    bool smm = ell > 0 && target > 0;
    qs.active_smm[q] = smm ? 1 : 0;
    if (!smm) {
        // AMC straight from e_s, e_t: max1 = 1, max2 = 0 for both vectors
        int32_t lf = ell;
        qs.lf[q] = lf;
        if (lf > 0) {
            double psi = psi_of(lf, 1.0, 0.0, 1.0, 0.0, ids, idt);
            double es = eta_star_of(psi, eps, tau, delta);
            qs.psi[q] = psi;
            qs.eta_star[q] = es;
            qs.eta1[q] = eta1_of(es, tau);
            qs.active_amc[q] = qs.eta1[q] > 0 ? 1 : 0;
            qs.stop[q] = GEER_STOP_CAP;
        } else {
            qs.active_amc[q] = 0;
            qs.stop[q] = GEER_STOP_NO_WALKS;
        }
    } else {
        qs.lf[q] = ell;
        qs.active_amc[q] = 0;
        qs.stop[q] = GEER_STOP_NO_WALKS;
    }
}

geer_status launch_init_queries(geer_graph *g, const QueryCtx &c, const int32_t *d_fixed,
                                int32_t forced_hops, hipStream_t st)
{
    if (c.nq == 0) return GEER_OK;
    int blocks = (int)((c.nq + 255) / 256);
    hipLaunchKernelGGL(k_init_queries, dim3(blocks), dim3(256), 0, st, c.qs, c.nq, g->d_row_ptr,
                       g->n, c.lambda, c.delta, c.tau, c.schedule, d_fixed, forced_hops,
                       c.ell_rule);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// hop 1: sparse scatter of P e_u into the (all-zero) H1 buffer; with
// `clear` the same positions are reset to zero instead.
// One wavefront per column (pair j, side).
// ----------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(64) void k_hop1(QState qs, SlotArgs sa,
                                             const int32_t *__restrict__ row_ptr,
                                             const int32_t *__restrict__ col_idx,
                                             const T *__restrict__ inv_deg, int clear)
{
    const int c = blockIdx.x;  // column within the batch
    const int k = blockIdx.y;  // batch (slot) within the group
    const int j = c >> 1, side = c & 1;
    if (j >= slot_nb(sa, k)) return;
    const int64_t q = qs.ord[slot_q0(sa, k) + j];
    const int lane = threadIdx.x;
    if (!clear && !qs.active_smm[q]) return;
    if (clear && qs.lb[q] < 1) return;  // hop 1 never ran for this pair
    T *h1 = slot_buf<T>(sa, k, 0);
    uint32_t *h1_bits = slot_bits(sa, k, 0);
    double *cs_m1 = slot_cs(sa, k), *cs_m2 = cs_m1 + kCols;
    int64_t *cs_sd = reinterpret_cast<int64_t *>(cs_m2 + kCols);
    const int32_t u = side ? qs.t[q] : qs.s[q];
    const int32_t b = row_ptr[u], e = row_ptr[u + 1];
    const uint32_t bit = 1u << (c & 31);
    T m1 = 0, m2 = 0;
    int64_t sd = 0;
    for (int32_t k = b + lane; k < e; k += 64) {
        int32_t v = col_idx[k];
        T val = inv_deg[v];
        size_t off = (size_t)v * kCols + c;
        uint32_t *bw = h1_bits + (size_t)v * kBitWords + (c >> 5);
        if (clear) {
            h1[off] = T(0);
            atomicAnd(bw, ~bit);
        } else {
            h1[off] = val;
            atomicOr(bw, bit);
            top2_push(m1, m2, val);
            sd += row_ptr[v + 1] - row_ptr[v];
        }
    }
    if (clear) return;
    // wavefront reduction of (max1, max2, degree sum)
    for (int o = 32; o > 0; o >>= 1) {
        T o1 = __shfl_xor(m1, o), o2 = __shfl_xor(m2, o);
        int64_t osd = __shfl_xor(sd, o);
        top2_push(m1, m2, o1);
        top2_push(m1, m2, o2);
        sd += osd;
    }
    if (lane == 0) {
        cs_m1[c] = (double)m1;
        cs_m2[c] = (double)m2;  // the zero entries (e.g. u itself) make max2 >= 0 exact
        cs_sd[c] = sd;
    }
}

// ----------------------------------------------------------------------------
// dense hop: gather over a range of CSR entries into per-lane accumulators
// ----------------------------------------------------------------------------

// A segment's sum has one fixed shape whatever the column tile: four
// interleaved partial sums S_j over the entries i = j mod 4 (in increasing i),
// combined as (S0 + S1) + (S2 + S3).  With NS = 64 / (KT/2) neighbour slots
// per wavefront, slot `slot` takes the entries i = slot mod NS and keeps the
// 4/NS partial sums S_slot, S_(slot+NS), ... in acc[].  The result of a
// heavy row is therefore bit-identical for every column tile, so the tile
// the autotuner picks from timings never changes an answer.
template <class T, int KT>
__device__ __forceinline__ void gather_range(const int32_t *__restrict__ col_idx,
                                             const T *__restrict__ in,
                                             const uint32_t *__restrict__ in_bits, int32_t b,
                                             int32_t e, int lane, int slot, int col, int bw,
                                             typename Vec2<T>::type (&acc)[4 / (64 / (KT / 2))],
                                             uint32_t &bacc)
{
    using T2 = typename Vec2<T>::type;
    constexpr int LPR = KT / 2;
    constexpr int NS = 64 / LPR;
    constexpr int A = 4 / NS;
    constexpr int U = 8;
    static_assert(U % A == 0 && 64 % (U * NS) == 0, "entry classes must stay fixed per accumulator");
    // Every lane runs the same trip counts so that the index broadcasts
    // (cross-lane reads) always execute with the whole wavefront active.
    for (int32_t base = b; base < e; base += 64) {
        const int cnt = min(64, e - base);
        const int32_t myidx = lane < cnt ? col_idx[base + lane] : 0;
        for (int k0 = 0; k0 < cnt; k0 += U * NS) {
            int32_t u[U];
            bool ok[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
                const int kk = k0 + i * NS + slot;
                ok[i] = kk < cnt;
                u[i] = __shfl(myidx, ok[i] ? kk : 0);
            }
            // support bits first: a pair whose two bits are clear at u has
            // exact zeros there, so its values are not fetched (whole lines
            // of the vector are skipped when none of their pairs reach u)
            uint32_t w[U];
#pragma unroll
            for (int i = 0; i < U; ++i) w[i] = ok[i] ? in_bits[(size_t)u[i] * kBitWords + bw] : 0u;
            T2 x[U];
#pragma unroll
            for (int i = 0; i < U; ++i) {
                if ((w[i] >> (col & 31)) & 3u) {
                    x[i] = *reinterpret_cast<const T2 *>(in + (size_t)u[i] * kCols + col);
                } else {
                    x[i].x = T(0);
                    x[i].y = T(0);
                }
            }
            // entry k0 + i*NS + slot lies in class (i*NS + slot) mod 4, i.e.
            // partial sum i mod A of this slot
#pragma unroll
            for (int i = 0; i < U; ++i) {
                acc[i % A].x += x[i].x;
                acc[i % A].y += x[i].y;
                bacc |= w[i];
            }
        }
    }
}

// Combine the partial sums of the NS neighbour slots into slot 0 as
// (S0 + S1) + (S2 + S3).
template <class T, int KT>
__device__ __forceinline__ typename Vec2<T>::type
reduce_slots(typename Vec2<T>::type (&acc)[4 / (64 / (KT / 2))], uint32_t &bacc)
{
    using T2 = typename Vec2<T>::type;
    constexpr int LPR = KT / 2;
    constexpr int NS = 64 / LPR;
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) bacc |= __shfl_xor(bacc, o);
    T2 r;
    if constexpr (NS == 4) {
        // slot j holds S_j: (S0 + S1) at slot 0 and (S2 + S3) at slot 2, then both
        T2 a = acc[0];
        a.x += __shfl_xor(a.x, LPR);
        a.y += __shfl_xor(a.y, LPR);
        a.x += __shfl_xor(a.x, 2 * LPR);
        a.y += __shfl_xor(a.y, 2 * LPR);
        r = a;
    } else if constexpr (NS == 2) {
        // slot 0 holds S0, S2; slot 1 holds S1, S3
        T2 p = acc[0], q = acc[1];
        p.x += __shfl_xor(p.x, LPR);
        p.y += __shfl_xor(p.y, LPR);
        q.x += __shfl_xor(q.x, LPR);
        q.y += __shfl_xor(q.y, LPR);
        r.x = p.x + q.x;
        r.y = p.y + q.y;
    } else {
        r.x = (acc[0].x + acc[1].x) + (acc[2].x + acc[3].x);
        r.y = (acc[0].y + acc[1].y) + (acc[2].y + acc[3].y);
    }
    return r;
}

// Write one finished row: values (active pairs only; a stopped pair's vectors
// may live in this buffer), the support word, and the per-lane statistics.
template <class T, int KT>
__device__ __forceinline__ void emit_row(T *__restrict__ out, uint32_t *__restrict__ out_bits,
                                         int32_t v, int32_t deg, T idg,
                                         const typename Vec2<T>::type &acc, uint32_t bacc,
                                         int lane, int slot, int col, int bw, bool act, T &m1s,
                                         T &m2s, T &m1t, T &m2t, uint32_t &sds, uint32_t &sdt)
{
    using T2 = typename Vec2<T>::type;
    const int bsh = col & 31;
    uint32_t mine = act ? ((bacc >> bsh) & 3u) : 0u;
    uint32_t word = mine << bsh;
    // OR the 16 lanes that share this support word (32 columns)
#pragma unroll
    for (int o = 1; o < 16; o <<= 1) word |= __shfl_xor(word, o);
    if (slot == 0) {
        T2 y;
        y.x = acc.x * idg;
        y.y = acc.y * idg;
        if (act) {
            *reinterpret_cast<T2 *>(out + (size_t)v * kCols + col) = y;
            top2_push(m1s, m2s, y.x);
            top2_push(m1t, m2t, y.y);
            if (mine & 1u) sds += (uint32_t)deg;
            if (mine & 2u) sdt += (uint32_t)deg;
        }
        if ((lane & 15) == 0) out_bits[(size_t)v * kBitWords + bw] = word;
    }
}

// Per-block reduction of the lane statistics, written to the partials at row `prow`.
template <class T, int KT>
__device__ __forceinline__ void write_block_stats(int lane, int wave, int slot, int col, T m1s,
                                                  T m2s, T m1t, T m2t, uint32_t sds,
                                                  uint32_t sdt, size_t prow,
                                                  double *__restrict__ p_m1,
                                                  double *__restrict__ p_m2,
                                                  int64_t *__restrict__ p_sd)
{
    constexpr int LPR = KT / 2;
    constexpr int NW = 4;
    __shared__ T s_m1[NW][KT], s_m2[NW][KT];
    __shared__ uint32_t s_sd[NW][KT];
    if (slot == 0) {
        const int cl = lane % LPR;
        s_m1[wave][2 * cl] = m1s;
        s_m2[wave][2 * cl] = m2s;
        s_m1[wave][2 * cl + 1] = m1t;
        s_m2[wave][2 * cl + 1] = m2t;
        s_sd[wave][2 * cl] = sds;
        s_sd[wave][2 * cl + 1] = sdt;
    }
    __syncthreads();
    const int col0 = col - 2 * (lane % LPR);
    for (int c = threadIdx.x; c < KT; c += blockDim.x) {
        T a1 = s_m1[0][c], a2 = s_m2[0][c];
        int64_t sd = s_sd[0][c];
        for (int w = 1; w < NW; ++w) {
            top2_push(a1, a2, s_m1[w][c]);
            top2_push(a1, a2, s_m2[w][c]);
            sd += s_sd[w][c];
        }
        size_t o = prow * kCols + col0 + c;
        p_m1[o] = (double)a1;
        p_m2[o] = (double)a2;
        p_sd[o] = sd;
    }
}

// Light rows: a group of KT/2 lanes owns one row (one column pair per lane),
// so a wavefront has 64/(KT/2) rows in flight.  Trip counts are uniform over
// the wavefront (the largest degree of its rows), so the index broadcasts
// always run with every lane active.
template <class T, int KT>
__global__ __launch_bounds__(256, (KT == 128 && sizeof(T) == 4) ? 8 : 5) void k_hop_light(
    const int32_t *__restrict__ row_ptr, const int32_t *__restrict__ col_idx,
    const T *__restrict__ inv_deg, const int32_t *__restrict__ rows, int32_t nrows,
    const T *__restrict__ in, T *__restrict__ out, const uint32_t *__restrict__ in_bits,
    uint32_t *__restrict__ out_bits, const uint64_t *__restrict__ mask_p, int col0,
    double *__restrict__ p_m1, double *__restrict__ p_m2, int64_t *__restrict__ p_sd)
{
    using T2 = typename Vec2<T>::type;
    constexpr int LPR = KT / 2;
    constexpr int RPW = 64 / LPR;
    constexpr int U = 8;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int grp = lane / LPR, li = lane % LPR;
    const int col = col0 + 2 * li;
    const int bw = col >> 5, bsh = col & 31;
    const bool act = ((*mask_p) >> (col >> 1)) & 1ull;
    T m1s = 0, m2s = 0, m1t = 0, m2t = 0;
    uint32_t sds = 0, sdt = 0;
    const int64_t stride = (int64_t)gridDim.x * 4 * RPW;
    for (int64_t r0 = ((int64_t)blockIdx.x * 4 + wave) * RPW; r0 < nrows; r0 += stride) {
        const int64_t r = r0 + grp;
        const bool has = r < nrows;
        const int32_t v = has ? rows[r] : 0;
        const int32_t b = has ? row_ptr[v] : 0;
        const int32_t d = has ? row_ptr[v + 1] - b : 0;
        int32_t dmax = d;
#pragma unroll
        for (int o = LPR; o < 64; o <<= 1) dmax = max(dmax, __shfl_xor(dmax, o));
        T2 acc;
        acc.x = T(0);
        acc.y = T(0);
        uint32_t bacc = 0;
        for (int32_t k0 = 0; k0 < dmax; k0 += LPR) {
            const int32_t myidx = (k0 + li < d) ? col_idx[b + k0 + li] : 0;
            for (int kk = 0; kk < LPR && k0 + kk < dmax; kk += U) {
                int32_t u[U];
                bool ok[U];
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    ok[i] = k0 + kk + i < d;
                    u[i] = __shfl(myidx, grp * LPR + kk + i);
                }
                // support bits first; clear bits mean exact zeros (not fetched)
                uint32_t w[U];
#pragma unroll
                for (int i = 0; i < U; ++i) w[i] = ok[i] ? in_bits[(size_t)u[i] * kBitWords + bw] : 0u;
                T2 x[U];
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    if ((w[i] >> (col & 31)) & 3u) {
                        x[i] = *reinterpret_cast<const T2 *>(in + (size_t)u[i] * kCols + col);
                    } else {
                        x[i].x = T(0);
                        x[i].y = T(0);
                    }
                }
#pragma unroll
                for (int i = 0; i < U; ++i) {
                    acc.x += x[i].x;
                    acc.y += x[i].y;
                    bacc |= w[i];
                }
            }
        }
        // emit the row of this group
        const uint32_t mine = (act && has) ? ((bacc >> bsh) & 3u) : 0u;
        uint32_t word = mine << bsh;
#pragma unroll
        for (int o = 1; o < 16; o <<= 1) word |= __shfl_xor(word, o);
        if (has) {
            const T idg = inv_deg[v];
            if (act) {
                T2 y;
                y.x = acc.x * idg;
                y.y = acc.y * idg;
                *reinterpret_cast<T2 *>(out + (size_t)v * kCols + col) = y;
                top2_push(m1s, m2s, y.x);
                top2_push(m1t, m2t, y.y);
                if (mine & 1u) sds += (uint32_t)d;
                if (mine & 2u) sdt += (uint32_t)d;
            }
            if ((li & 15) == 0) out_bits[(size_t)v * kBitWords + bw] = word;
        }
    }
    // merge the statistics of the row groups (disjoint row sets) into group 0
#pragma unroll
    for (int o = LPR; o < 64; o <<= 1) {
        T a1 = __shfl_xor(m1s, o), a2 = __shfl_xor(m2s, o);
        T b1 = __shfl_xor(m1t, o), b2 = __shfl_xor(m2t, o);
        uint32_t c1 = __shfl_xor(sds, o), c2 = __shfl_xor(sdt, o);
        top2_push(m1s, m2s, a1);
        top2_push(m1s, m2s, a2);
        top2_push(m1t, m2t, b1);
        top2_push(m1t, m2t, b2);
        sds += c1;
        sdt += c2;
    }
    write_block_stats<T, KT>(lane, wave, grp, col, m1s, m2s, m1t, m2t, sds, sdt, blockIdx.x, p_m1,
                             p_m2, p_sd);
}

// Heavy rows, pass 1: partial sums of 256-entry segments.
template <class T, int KT>
__global__ __launch_bounds__(256) void k_hop_segments(
    const int32_t *__restrict__ col_idx, const int32_t *__restrict__ seg_b,
    const int32_t *__restrict__ seg_e, int32_t nseg, const T *__restrict__ in,
    const uint32_t *__restrict__ in_bits, T *__restrict__ segbuf, uint32_t *__restrict__ segbits,
    int col0)
{
    using T2 = typename Vec2<T>::type;
    constexpr int LPR = KT / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / LPR;
    const int col = col0 + 2 * (lane % LPR);
    const int bw = col >> 5;
    for (int32_t sgi = blockIdx.x * 4 + wave; sgi < nseg; sgi += gridDim.x * 4) {
        T2 parts[4 / (64 / LPR)];
#pragma unroll
        for (int a = 0; a < 4 / (64 / LPR); ++a) parts[a].x = parts[a].y = T(0);
        uint32_t bacc = 0;
        gather_range<T, KT>(col_idx, in, in_bits, seg_b[sgi], seg_e[sgi], lane, slot, col, bw,
                            parts, bacc);
        const T2 acc = reduce_slots<T, KT>(parts, bacc);
        if (slot == 0) {
            *reinterpret_cast<T2 *>(segbuf + (size_t)sgi * kCols + col) = acc;
            if ((lane & 15) == 0) segbits[(size_t)sgi * kBitWords + bw] = bacc;
        }
    }
}

// Heavy rows, pass 2: sum the segments of each row in order, then emit.
template <class T, int KT>
__global__ __launch_bounds__(256) void k_hop_heavy_fin(
    const int32_t *__restrict__ row_ptr, const T *__restrict__ inv_deg,
    const int32_t *__restrict__ heavy_rows, const int32_t *__restrict__ seg_start, int32_t nheavy,
    const T *__restrict__ segbuf, const uint32_t *__restrict__ segbits, T *__restrict__ out,
    uint32_t *__restrict__ out_bits, const uint64_t *__restrict__ mask_p, int col0,
    size_t prow0, double *__restrict__ p_m1, double *__restrict__ p_m2,
    int64_t *__restrict__ p_sd)
{
    using T2 = typename Vec2<T>::type;
    constexpr int LPR = KT / 2;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int slot = lane / LPR;
    const int col = col0 + 2 * (lane % LPR);
    const int bw = col >> 5;
    const bool act = ((*mask_p) >> (col >> 1)) & 1ull;
    T m1s = 0, m2s = 0, m1t = 0, m2t = 0;
    uint32_t sds = 0, sdt = 0;
    for (int32_t h = blockIdx.x * 4 + wave; h < nheavy; h += gridDim.x * 4) {
        const int32_t v = heavy_rows[h];
        T2 acc;
        acc.x = T(0);
        acc.y = T(0);
        uint32_t bacc = 0;
        if (slot == 0) {
            for (int32_t sg = seg_start[h]; sg < seg_start[h + 1]; ++sg) {
                T2 x = *reinterpret_cast<const T2 *>(segbuf + (size_t)sg * kCols + col);
                acc.x += x.x;
                acc.y += x.y;
                bacc |= segbits[(size_t)sg * kBitWords + bw];
            }
        }
        emit_row<T, KT>(out, out_bits, v, row_ptr[v + 1] - row_ptr[v], inv_deg[v], acc, bacc,
                        lane, slot, col, bw, act, m1s, m2s, m1t, m2t, sds, sdt);
    }
    write_block_stats<T, KT>(lane, wave, slot, col, m1s, m2s, m1t, m2t, sds, sdt,
                             prow0 + blockIdx.x, p_m1, p_m2, p_sd);
}

// Column statistics: reduce the per-block partials of every active column.
__global__ __launch_bounds__(256) void k_colstat_reduce(const double *__restrict__ p_m1,
                                                        const double *__restrict__ p_m2,
                                                        const int64_t *__restrict__ p_sd,
                                                        int nrows_part,
                                                        const uint64_t *__restrict__ mask_p,
                                                        double *__restrict__ cs_m1,
                                                        double *__restrict__ cs_m2,
                                                        int64_t *__restrict__ cs_sd)
{
    const int c = blockIdx.x;
    if (!(((*mask_p) >> (c >> 1)) & 1ull)) return;
    double a1 = 0.0, a2 = 0.0;
    int64_t sd = 0;
    for (int r = threadIdx.x; r < nrows_part; r += blockDim.x) {
        size_t o = (size_t)r * kCols + c;
        top2_push(a1, a2, p_m1[o]);
        top2_push(a1, a2, p_m2[o]);
        sd += p_sd[o];
    }
    __shared__ double s1[256], s2[256];
    __shared__ int64_t ss[256];
    s1[threadIdx.x] = a1;
    s2[threadIdx.x] = a2;
    ss[threadIdx.x] = sd;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double b1 = s1[threadIdx.x], b2 = s2[threadIdx.x];
            top2_push(b1, b2, s1[threadIdx.x + w]);
            top2_push(b1, b2, s2[threadIdx.x + w]);
            s1[threadIdx.x] = b1;
            s2[threadIdx.x] = b2;
            ss[threadIdx.x] += ss[threadIdx.x + w];
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cs_m1[c] = s1[0];
        cs_m2[c] = s2[0];
        cs_sd[c] = ss[0];
    }
}

// Hop-2 column statistics of a group: the `split` partial rows of each
// column of a pair in the slot's hop-2 mask.  One wavefront per (column, slot).
__global__ __launch_bounds__(64) void k_colstat_group(SlotArgs sa, int split)
{
    const int c = blockIdx.x, k = blockIdx.y, lane = threadIdx.x;
    if (!((sa.meta[sa.G + k] >> (c >> 1)) & 1ull)) return;
    const double *hp = slot_hpart(sa, k);
    const int64_t *hsd = reinterpret_cast<const int64_t *>(hp + 2 * kPushSplitMax * kCols);
    double a1 = 0.0, a2 = 0.0;
    int64_t sd = 0;
    if (lane < split) {
        const size_t o = (size_t)lane * kCols + c;
        a1 = hp[o];
        a2 = hp[kPushSplitMax * kCols + o];
        sd = hsd[o];
    }
    for (int o = 32; o > 0; o >>= 1) {
        const double b1 = __shfl_xor(a1, o), b2 = __shfl_xor(a2, o);
        top2_push(a1, a2, b1);
        top2_push(a1, a2, b2);
        sd += __shfl_xor(sd, o);
    }
    if (lane == 0) {
        double *cs = slot_cs(sa, k);
        cs[c] = a1;
        cs[kCols + c] = a2;
        reinterpret_cast<int64_t *>(cs + 2 * kCols)[c] = sd;
    }
}

int grid_blocks_dense(const geer_graph *g) { return std::max(1, g->num_cus * 8); }

static int heavy_fin_blocks(const geer_graph *g)
{
    return std::max(1, std::min(g->num_cus * 2, (g->n_heavy + 3) / 4));
}

template <class T, int KT>
static geer_status hop_dense_t(geer_graph *g, const HopArgs &a, hipStream_t st)
{
    Workspace &ws = g->ws;
    const int nb = grid_blocks_dense(g);
    const int nf = heavy_fin_blocks(g);
    const size_t prows = (size_t)nb + nf;
    double *p_m1 = ws.part.as<double>();
    double *p_m2 = p_m1 + prows * kCols;
    int64_t *p_sd = reinterpret_cast<int64_t *>(p_m2 + prows * kCols);
    const T *inv = std::is_same<T, float>::value ? (const T *)g->d_inv_deg_f
                                                 : (const T *)g->d_inv_deg_d;
    const T *in = (const T *)a.in;
    T *out = (T *)a.out;
    // algorithmic bytes of this tile (split over the three kernels):
    // 4(|R|+1) + 4 nnz(R) + b k |C| + b k |R| + 4 |R| with R = C = all rows and
    // k = active columns of the tile; the gathered-vector term is shared in
    // proportion to the CSR entries each kernel walks.
    int kact = 0;
    for (int j = a.col0 / 2; j < (a.col0 + KT) / 2; ++j) kact += (int)((a.host_mask >> j) & 1ull) * 2;
    const double b = (double)sizeof(T), n = (double)g->n, nnz = (double)g->nnz;
    const double nnz_h = (double)g->nnz_heavy, nnz_l = nnz - nnz_h;
    const double xread = b * kact * n;
    if (g->n_seg > 0) {
        T *segbuf = ws.segbuf.as<T>();
        uint32_t *segbits = reinterpret_cast<uint32_t *>(segbuf + (size_t)g->n_seg * kCols);
        int sb = std::max(1, std::min(nb, (g->n_seg + 3) / 4));
        int tok = prof_begin(g, st);
        hipLaunchKernelGGL((k_hop_segments<T, KT>), dim3(sb), dim3(256), 0, st, g->d_col_idx,
                           g->d_seg_begin, g->d_seg_end, g->n_seg, in, a.in_bits, segbuf, segbits,
                           a.col0);
        prof_end(g, tok, PK_HOP_SEGMENTS, 4.0 * nnz_h + xread * (nnz_h / nnz), nnz_h * kact, st);
        GEER_HIP(hipGetLastError());
    }
    {
        const double nl = (double)g->n_light;
        int tok = prof_begin(g, st);
        hipLaunchKernelGGL((k_hop_light<T, KT>), dim3(nb), dim3(256), 0, st, g->d_row_ptr,
                           g->d_col_idx, inv, g->d_light_rows, g->n_light, in, out, a.in_bits,
                           a.out_bits, a.mask, a.col0, p_m1, p_m2, p_sd);
        prof_end(g, tok, PK_HOP_LIGHT,
                 4.0 * (nl + 1) + 4.0 * nnz_l + xread * (nnz_l / nnz) + b * kact * nl + 4.0 * nl,
                 nnz_l * kact, st);
        GEER_HIP(hipGetLastError());
    }
    if (g->n_heavy > 0) {
        T *segbuf = ws.segbuf.as<T>();
        uint32_t *segbits = reinterpret_cast<uint32_t *>(segbuf + (size_t)g->n_seg * kCols);
        const double nh = (double)g->n_heavy;
        int tok = prof_begin(g, st);
        hipLaunchKernelGGL((k_hop_heavy_fin<T, KT>), dim3(nf), dim3(256), 0, st, g->d_row_ptr,
                           inv, g->d_heavy_rows, g->d_heavy_seg_start, g->n_heavy, segbuf,
                           segbits, out, a.out_bits, a.mask, a.col0, (size_t)nb, p_m1, p_m2,
                           p_sd);
        prof_end(g, tok, PK_HOP_HEAVY_FIN, 4.0 * (nh + 1) + b * kact * nh + 4.0 * nh, 0.0, st);
        GEER_HIP(hipGetLastError());
    } else {
        // keep the partial rows of the (absent) heavy pass neutral
        GEER_TRY(launch_zero(g, p_m1 + (size_t)nb * kCols, (size_t)nf * kCols * sizeof(double), st));
        GEER_TRY(launch_zero(g, p_m2 + (size_t)nb * kCols, (size_t)nf * kCols * sizeof(double), st));
        GEER_TRY(launch_zero(g, p_sd + (size_t)nb * kCols, (size_t)nf * kCols * sizeof(int64_t), st));
    }
    return GEER_OK;
}

geer_status reserve_dense(geer_graph *g, int value_size)
{
    Workspace &ws = g->ws;
    const size_t prows = (size_t)grid_blocks_dense(g) + heavy_fin_blocks(g);
    GEER_TRY(ws.part.reserve(prows * kCols * (2 * sizeof(double) + sizeof(int64_t))));
    GEER_TRY(ws.segbuf.reserve((size_t)std::max(g->n_seg, 1) *
                               (kCols * (size_t)value_size + kBitWords * sizeof(uint32_t))));
    return GEER_OK;
}

geer_status launch_hop_dense(geer_graph *g, const HopArgs &a, int value_size, hipStream_t st)
{
    Workspace &ws = g->ws;
    const int nb = grid_blocks_dense(g);
    const int nf = heavy_fin_blocks(g);
    const size_t prows = (size_t)nb + nf;
    GEER_TRY(reserve_dense(g, value_size));
    const int kt = a.col_tile;
    const int whole = prof_begin(g, st);
    for (int c0 = 0; c0 < kCols; c0 += kt) {
        // a tile without an active pair has nothing to compute (its columns
        // are not read again: stopped pairs keep their vectors elsewhere)
        const uint64_t tile_pairs = kt == 128 ? ~0ull : (((1ull << (kt / 2)) - 1ull) << (c0 / 2));
        if ((a.host_mask & tile_pairs) == 0) continue;
        HopArgs t = a;
        t.col0 = c0;
        geer_status s = GEER_E_INVALID_ARG;
        if (value_size == 4) {
            if (kt == 128) s = hop_dense_t<float, 128>(g, t, st);
            else if (kt == 64) s = hop_dense_t<float, 64>(g, t, st);
            else if (kt == 32) s = hop_dense_t<float, 32>(g, t, st);
        } else {
            if (kt == 128) s = hop_dense_t<double, 128>(g, t, st);
            else if (kt == 64) s = hop_dense_t<double, 64>(g, t, st);
            else if (kt == 32) s = hop_dense_t<double, 32>(g, t, st);
        }
        if (s != GEER_OK) return s == GEER_E_INVALID_ARG ? fail(s, "unsupported column tile") : s;
    }
    double *cs_m1 = a.cs;
    double *cs_m2 = cs_m1 + kCols;
    int64_t *cs_sd = reinterpret_cast<int64_t *>(cs_m2 + kCols);
    double *p_m1 = ws.part.as<double>();
    double *p_m2 = p_m1 + prows * kCols;
    int64_t *p_sd = reinterpret_cast<int64_t *>(p_m2 + prows * kCols);
    int tok = prof_begin(g, st);
    hipLaunchKernelGGL(k_colstat_reduce, dim3(kCols), dim3(256), 0, st, p_m1, p_m2, p_sd,
                       (int)prows, a.mask, cs_m1, cs_m2, cs_sd);
    prof_end(g, tok, PK_COLSTAT, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    prof_end(g, whole, PK_DENSE_HOP, 0.0, 1.0, st);
    return GEER_OK;
}

geer_status launch_hop1_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int nslots,
                              bool clear, hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    const dim3 grid(2 * sa.B, nslots);
    int tok = prof_begin(g, st);
    if (g->ws.value_size == 4)
        hipLaunchKernelGGL(k_hop1<float>, grid, dim3(64), 0, st, c.qs, sa, g->d_row_ptr,
                           g->d_col_idx, g->d_inv_deg_f, clear ? 1 : 0);
    else
        hipLaunchKernelGGL(k_hop1<double>, grid, dim3(64), 0, st, c.qs, sa, g->d_row_ptr,
                           g->d_col_idx, g->d_inv_deg_d, clear ? 1 : 0);
    prof_end(g, tok, PK_HOP1, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// Clear a profiler counter pair (device counts are added to it).
__global__ void k_zero_counter(int64_t *c)
{
    if (threadIdx.x < 2) c[threadIdx.x] = 0;
}

// Selective hop-1 scatter (modes in geer_internal.h).  Whether a pair's
// columns are written (or cleared) depends on its flag and its state only.
__device__ __forceinline__ bool hop1_need(const QState &qs, int64_t q, int mode,
                                          const int32_t *__restrict__ row_ptr)
{
    if (mode == kHop1Clear) return qs.h1w[q] != 0;
    if (qs.h1w[q] || qs.lb[q] != 1) return false;
    if (mode == kHop1Stopped) {
        // the walk kernel evaluates the vector from LDS rows when both rows fit
        const int32_t s = qs.s[q], t = qs.t[q];
        const int32_t ds = row_ptr[s + 1] - row_ptr[s], dt = row_ptr[t + 1] - row_ptr[t];
        return !qs.active_smm[q] && (ds > kMemberRowMax || dt > kMemberRowMax);
    }
    return qs.active_smm[q] != 0;
}

// The gridDim.y blocks of a slot share every selected pair's two rows: each
// of their wavefronts takes every (4 gridDim.y)-th run of 64 entries, so a hub
// row of 4e5 entries is scattered by hundreds of wavefronts at once.  The
// flags are only read here; k_hop1_flags updates them afterwards.  entries
// (nullable, for the profiler): CSR entries scattered, summed over the launch.

template <class T>
__global__ __launch_bounds__(256) void k_hop1_select(QState qs, SlotArgs sa, int slot0, int mode,
                                                     const int32_t *__restrict__ row_ptr,
                                                     const int32_t *__restrict__ col_idx,
                                                     const T *__restrict__ inv_deg,
                                                     unsigned long long *__restrict__ entries)
{
    const int k = slot0 + (int)blockIdx.x;
    const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
    const int nb = slot_nb(sa, k);
    const int64_t q0 = slot_q0(sa, k);
    const bool need = lane < nb && hop1_need(qs, qs.ord[q0 + lane], mode, row_ptr);
    uint64_t m = __ballot(need);
    const int gw = (int)blockIdx.y * 4 + wave, nw = (int)gridDim.y * 4;
    T *h1 = slot_buf<T>(sa, k, 0);
    uint32_t *h1_bits = slot_bits(sa, k, 0);
    int64_t cnt = 0;
    while (m) {
        const int j = __ffsll((unsigned long long)m) - 1;
        m &= m - 1;
        const int64_t q = qs.ord[q0 + j];
        for (int side = 0; side < 2; ++side) {
            const int c = 2 * j + side;
            const int32_t u = side ? qs.t[q] : qs.s[q];
            const uint32_t bit = 1u << (c & 31);
            const int32_t b = row_ptr[u], e1 = row_ptr[u + 1];
            cnt += e1 - b;
            for (int32_t e = b + gw * 64 + lane; e < e1; e += nw * 64) {
                const int32_t v = col_idx[e];
                uint32_t *bw = h1_bits + (size_t)v * kBitWords + (c >> 5);
                if (mode == kHop1Clear) {
                    h1[(size_t)v * kCols + c] = T(0);
                    atomicAnd(bw, ~bit);
                } else {
                    h1[(size_t)v * kCols + c] = inv_deg[v];
                    atomicOr(bw, bit);
                }
            }
        }
    }
    if (entries && gw == 0 && lane == 0 && cnt) atomicAdd(entries, (unsigned long long)cnt);
}

// The flags of the pairs k_hop1_select just wrote (set) or cleared (reset).
__global__ __launch_bounds__(64) void k_hop1_flags(QState qs, SlotArgs sa, int slot0, int mode,
                                                   const int32_t *__restrict__ row_ptr)
{
    const int k = slot0 + (int)blockIdx.x;
    const int j = threadIdx.x;
    if (j >= slot_nb(sa, k)) return;
    const int64_t q = qs.ord[slot_q0(sa, k) + j];
    if (hop1_need(qs, q, mode, row_ptr)) qs.h1w[q] = mode == kHop1Clear ? 0 : 1;
}

geer_status launch_hop1_select(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int slot0,
                               int nslots, int mode, hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    // profiled: CSR entries scattered, each a 4-byte index read, a value
    // written and a 4-byte support word updated
    int counter = -1;
    int64_t *d_cnt = prof_counter(g, &counter);
    int tok = prof_begin(g, st);
    unsigned long long *ent = reinterpret_cast<unsigned long long *>(d_cnt);
    if (d_cnt) hipLaunchKernelGGL(k_zero_counter, dim3(1), dim3(64), 0, st, d_cnt);
    // about 2048 blocks in all (8 per CU), at least 16 per slot
    const dim3 grid(nslots, std::max(16, std::min(512, 2048 / nslots)));
    if (g->ws.value_size == 4)
        hipLaunchKernelGGL(k_hop1_select<float>, grid, dim3(256), 0, st, c.qs, sa, slot0, mode,
                           g->d_row_ptr, g->d_col_idx, g->d_inv_deg_f, ent);
    else
        hipLaunchKernelGGL(k_hop1_select<double>, grid, dim3(256), 0, st, c.qs, sa, slot0, mode,
                           g->d_row_ptr, g->d_col_idx, g->d_inv_deg_d, ent);
    GEER_HIP(hipGetLastError());
    hipLaunchKernelGGL(k_hop1_flags, dim3(nslots), dim3(64), 0, st, c.qs, sa, slot0, mode, g->d_row_ptr);
    prof_end_counted(g, tok, PK_HOP1, counter, 8.0 + (double)g->ws.value_size, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// epilogue after a hop: r_b increment, switch rule, AMC parameters on stop
// ----------------------------------------------------------------------------

// 1/d rounded to the vector type, as the inverse-degree tables hold it
template <class T> __device__ __forceinline__ double inv_as(int32_t d)
{
    return (double)(T)(1.0 / (double)d);
}

template <class T>
__global__ void k_epilogue(QState qs, SlotArgs sa, int hop, int which,
                           const int32_t *__restrict__ row_ptr, int32_t schedule, int32_t tau,
                           double delta, int implicit1, const int32_t *__restrict__ col_idx,
                           const T *__restrict__ inv_deg, const int32_t *__restrict__ nbr_min,
                           const int32_t *__restrict__ nbr_deg2,
                           const int64_t *__restrict__ nbr_work)
{
    const int k = blockIdx.x;  // batch (slot) within the group
    const int j = threadIdx.x;
    if (j >= slot_nb(sa, k)) return;
    const int64_t q = qs.ord[slot_q0(sa, k) + j];
    if (!qs.active_smm[q]) return;
    const T *vec = slot_buf<T>(sa, k, which);
    const int64_t vec_elem_off = slot_elem_off(sa, k, which);
    const double *cs_m1 = slot_cs(sa, k), *cs_m2 = cs_m1 + kCols;
    const int64_t *cs_sd = reinterpret_cast<const int64_t *>(cs_m2 + kCols);
    uint64_t *mask = sa.meta + k;
    const int32_t s = qs.s[q], t = qs.t[q];
    const double ids = 1.0 / (row_ptr[s + 1] - row_ptr[s]);
    const double idt = 1.0 / (row_ptr[t + 1] - row_ptr[t]);
    const size_t cs = 2 * j, ct = 2 * j + 1;
    double xs, xt, ys, yt, m1s, m2s, m1t, m2t;
    int64_t sd;
    if (hop == 1 && implicit1) {
        // P e_s is 1/d(v) on N(s) and 0 elsewhere (no self-loops): it is 0 at
        // s, 1/d(t) at t when (s,t) is an edge; its two largest entries are
        // 1/d of the two smallest neighbour degrees; its support N(s) has
        // degree sum sum_{v in N(s)} d(v).  Same for t.
        int32_t lo = row_ptr[s], hi = row_ptr[s + 1];
        const int32_t end = hi;
        while (lo < hi) {
            const int32_t mid = (lo + hi) >> 1;
            if (col_idx[mid] < t) lo = mid + 1;
            else hi = mid;
        }
        const bool edge = lo < end && col_idx[lo] == t;
        xs = 0.0;
        yt = 0.0;
        xt = edge ? (double)inv_deg[t] : 0.0;
        ys = edge ? (double)inv_deg[s] : 0.0;
        m1s = inv_as<T>(nbr_min[s]);
        m2s = nbr_deg2[s] > 0 ? inv_as<T>(nbr_deg2[s]) : 0.0;
        m1t = inv_as<T>(nbr_min[t]);
        m2t = nbr_deg2[t] > 0 ? inv_as<T>(nbr_deg2[t]) : 0.0;
        sd = nbr_work[s] + nbr_work[t];
    } else {
        xs = (double)vec[(size_t)s * kCols + cs];
        xt = (double)vec[(size_t)t * kCols + cs];
        ys = (double)vec[(size_t)s * kCols + ct];
        yt = (double)vec[(size_t)t * kCols + ct];
        m1s = cs_m1[cs];
        m2s = cs_m2[cs];
        m1t = cs_m1[ct];
        m2t = cs_m2[ct];
        sd = cs_sd[cs] + cs_sd[ct];
    }
    // Algorithm 2: r_b += s*(s)/d(s) + t*(t)/d(t) - s*(t)/d(s) - t*(s)/d(t)
    const double rb = qs.rb[q] + (xs * ids + yt * idt - xt * ids - ys * idt);
    qs.rb[q] = rb;
    qs.lb[q] = hop;
    const int32_t ell = qs.ell[q];
    const int32_t lf = ell - hop;
    const double eps = qs.eps[q];
    tau = qs.tau_q[q];  // per-pair batch count (the learned schedule may set it)
    const double psi = psi_of(lf, m1s, m2s, m1t, m2t, ids, idt);
    const double es = eta_star_of(psi, eps, tau, delta);
    const int64_t e1 = eta1_of(es, tau);
    bool stop = hop >= qs.lb_target[q];
    if (!stop && (schedule == GEER_SCHEDULE_GREEDY || qs.fallback[q])) {
        // Eq. (smm-amc): next-hop cost sum_{V_s} d + sum_{V_t} d versus h(l - l_b)
        const double h = (ldexp(1.0, tau) - 1.0) * (double)e1;
        stop = (double)sd > h;
    }
    if (stop) {
        qs.active_smm[q] = 0;
        qs.lf[q] = lf;
        qs.supp_sum[q] = sd;
        qs.vec_off[q] = vec_elem_off + 2 * j;
        qs.psi[q] = lf > 0 ? psi : 0.0;
        qs.eta_star[q] = lf > 0 ? es : 0.0;
        qs.eta1[q] = lf > 0 ? e1 : 0;
        qs.active_amc[q] = (lf > 0 && e1 > 0) ? 1 : 0;
        qs.stop[q] = lf > 0 ? GEER_STOP_CAP : GEER_STOP_NO_WALKS;
        atomicAnd(reinterpret_cast<unsigned long long *>(mask), ~(1ull << j));
    }
}

geer_status launch_epilogue_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa,
                                  int nslots, int hop, int which, int value_size, hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    int tok = prof_begin(g, st);
    const int imp = c.hop1_implicit ? 1 : 0;
    if (value_size == 4)
        hipLaunchKernelGGL(k_epilogue<float>, dim3(nslots), dim3(64), 0, st, c.qs, sa, hop, which,
                           g->d_row_ptr, c.schedule, c.tau, c.delta, imp, g->d_col_idx,
                           g->d_inv_deg_f, g->d_min_nbr_deg, g->d_nbr_deg2, g->d_nbr_work);
    else
        hipLaunchKernelGGL(k_epilogue<double>, dim3(nslots), dim3(64), 0, st, c.qs, sa, hop, which,
                           g->d_row_ptr, c.schedule, c.tau, c.delta, imp, g->d_col_idx,
                           g->d_inv_deg_d, g->d_min_nbr_deg, g->d_nbr_deg2, g->d_nbr_work);
    prof_end(g, tok, PK_EPILOGUE, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// ----------------------------------------------------------------------------
// Largest / second-largest of the first `ncols` columns of a slot buffer
// (used when AMC is given caller vectors).  One block per column.
// ----------------------------------------------------------------------------

template <class T>
__global__ __launch_bounds__(256) void k_column_top2(const T *__restrict__ vec, int32_t n,
                                                     int stride, double *__restrict__ cs_m1,
                                                     double *__restrict__ cs_m2)
{
    const int c = blockIdx.x;
    T a1 = 0, a2 = 0;
    for (int32_t v = threadIdx.x; v < n; v += blockDim.x) top2_push(a1, a2, vec[(size_t)v * stride + c]);
    __shared__ double s1[256], s2[256];
    s1[threadIdx.x] = (double)a1;
    s2[threadIdx.x] = (double)a2;
    __syncthreads();
    for (int w = 128; w > 0; w >>= 1) {
        if ((int)threadIdx.x < w) {
            double b1 = s1[threadIdx.x], b2 = s2[threadIdx.x];
            top2_push(b1, b2, s1[threadIdx.x + w]);
            top2_push(b1, b2, s2[threadIdx.x + w]);
            s1[threadIdx.x] = b1;
            s2[threadIdx.x] = b2;
        }
        __syncthreads();
    }
    if (threadIdx.x == 0) {
        cs_m1[c] = s1[0];
        cs_m2[c] = s2[0];
    }
}

geer_status launch_column_top2(const geer_graph *g, const void *vec, int ncols, int stride,
                               int value_size, double *cs_m1, double *cs_m2, hipStream_t st)
{
    if (value_size == 4)
        hipLaunchKernelGGL(k_column_top2<float>, dim3(ncols), dim3(256), 0, st,
                           (const float *)vec, g->n, stride, cs_m1, cs_m2);
    else
        hipLaunchKernelGGL(k_column_top2<double>, dim3(ncols), dim3(256), 0, st,
                           (const double *)vec, g->n, stride, cs_m1, cs_m2);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

}  // namespace geer

namespace geer {

// ----------------------------------------------------------------------------
// Sparse hop 2 (push from the hop-1 frontier).  After one product the vector
// of column c is x1(v) = 1/d(v) on N(u) (u = s or t), so
//     x2(w) = (1/d(w)) * sum_{v in N(u), w in N(v)} 1/d(v).
// The work is sum_{v in N(u)} d(v) instead of a pass over the whole graph.
// Contributions are added as unsigned fixed point (1/d(v) * 2^F rounded once
// per v) with integer atomics, so every sum is exact and independent of the
// order of the additions; the first visitor of an entry takes the sum with an
// exchange (which also resets the accumulator to zero), scales it by 1/d(w)
// in FP64, rounds once to the vector type and records the statistics.
// ----------------------------------------------------------------------------

__device__ __forceinline__ unsigned long long fixed_inv_deg(double inv_d, int shift)
{
    return __double2ull_rn(ldexp(inv_d, shift));
}

constexpr int kPushChunk = 2048;  // neighbours of u staged in LDS per round

// mode 0: accumulate; mode 1: convert + stats; mode 2: clear the output entries.
// The work of column c is the concatenation of the rows N(v), v in N(u),
// shared by the column's `split` blocks.  A block stages a chunk of N(u) and
// the prefix sums of the degrees in LDS and spreads the chunk's flattened
// entries over its lanes.  When N(u) has at least `split` chunks, each block
// takes whole chunks (every split-th); otherwise every block stages every
// chunk and takes every split-th run of 256 entries.  Either way a hub
// column is spread over all its blocks, and no result depends on the split
// (sums are exact integers, each entry is converted by its first visitor).
template <class T, int MODE>
__global__ __launch_bounds__(256) void k_hop2_sparse(
    QState qs, SlotArgs sa, int slot0, const int32_t *__restrict__ row_ptr,
    const int32_t *__restrict__ col_idx, const double *__restrict__ inv_deg_d,
    unsigned long long *__restrict__ acc, int shift, int split)
{
    __shared__ int32_t s_v[kPushChunk];
    __shared__ int32_t s_beg[kPushChunk];
    __shared__ int32_t s_pre[kPushChunk + 1];
    __shared__ int32_t s_tmp[256];
    const int c = blockIdx.x;
    const int slot = slot0 + (int)blockIdx.y / split;
    const int k = (int)blockIdx.y % split;  // this block's share of the column
    const int j = c >> 1;
    // modes 0/1: per-column global-path mask (two words); mode 2: the pair mask
    const uint64_t *mask_p = MODE == 2 ? sa.meta + sa.G + slot : sa.meta + 2 * sa.G + 4 * slot + 2;
    const bool act = MODE == 2 ? (((*mask_p) >> j) & 1ull) : ((mask_p[c >> 6] >> (c & 63)) & 1ull);
    T *out = slot_buf<T>(sa, slot, 1);
    uint32_t *out_bits = slot_bits(sa, slot, 1);
    unsigned long long *acc_s = acc + (size_t)(slot - slot0) * sa.buf_elems;
    const int tid = threadIdx.x;
    const int lane = tid & 63, wave = tid >> 6;
    T m1 = 0, m2 = 0;
    int64_t sd = 0;
    if (act) {
        const int64_t q = qs.ord[slot_q0(sa, slot) + j];
        const int32_t u = (c & 1) ? qs.t[q] : qs.s[q];
        const int32_t b0 = row_ptr[u], du = row_ptr[u + 1] - b0;
        const uint32_t bit = 1u << (c & 31);
        const int32_t nch = (du + kPushChunk - 1) / kPushChunk;
        const bool by_chunk = nch >= split;
        for (int32_t ch = by_chunk ? k : 0; ch < nch; ch += by_chunk ? split : 1) {
            const int32_t base = ch * kPushChunk;
            const int cnt = min(kPushChunk, du - base);
            // stage v, its row start and degree; 256-thread scan of the degrees
            const int per = (cnt + 255) / 256;
            int32_t local = 0;
            for (int i = tid * per; i < min(cnt, (tid + 1) * per); ++i) {
                const int32_t v = col_idx[b0 + base + i];
                const int32_t rb = row_ptr[v];
                s_v[i] = v;
                s_beg[i] = rb;
                s_pre[i] = row_ptr[v + 1] - rb;  // degree for now
                local += s_pre[i];
            }
            s_tmp[tid] = local;
            __syncthreads();
            for (int o = 1; o < 256; o <<= 1) {
                int32_t add = tid >= o ? s_tmp[tid - o] : 0;
                __syncthreads();
                s_tmp[tid] += add;
                __syncthreads();
            }
            int32_t run = s_tmp[tid] - local;
            for (int i = tid * per; i < min(cnt, (tid + 1) * per); ++i) {
                const int32_t d = s_pre[i];
                s_pre[i] = run;
                run += d;
            }
            if (tid == 255) s_pre[cnt] = s_tmp[255];
            __syncthreads();
            const int32_t total = s_pre[cnt];
            const int32_t p0 = by_chunk ? tid : k * 256 + tid;
            const int32_t pstep = by_chunk ? 256 : split * 256;
            for (int32_t p = p0; p < total; p += pstep) {
                // entry p lies in row s_v[i] with s_pre[i] <= p < s_pre[i+1]
                int lo = 0, hi = cnt;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const int32_t v = s_v[lo];
                const int32_t w = col_idx[s_beg[lo] + (p - s_pre[lo])];
                const size_t off = (size_t)w * kCols + c;
                if (MODE == 0) {
                    atomicAdd(acc_s + off, fixed_inv_deg(inv_deg_d[v], shift));
                } else if (MODE == 1) {
                    const unsigned long long tot = atomicExch(acc_s + off, 0ull);
                    if (tot != 0ull) {
                        const T val = (T)(ldexp((double)tot, -shift) * inv_deg_d[w]);
                        out[off] = val;
                        atomicOr(out_bits + (size_t)w * kBitWords + (c >> 5), bit);
                        top2_push(m1, m2, val);
                        sd += row_ptr[w + 1] - row_ptr[w];
                    }
                } else {
                    out[off] = T(0);
                    atomicAnd(out_bits + (size_t)w * kBitWords + (c >> 5), ~bit);
                }
            }
            __syncthreads();
        }
    }
    if (MODE != 1 || !act) return;
    // block reduction of the statistics -> partial row k of column c
    for (int o = 32; o > 0; o >>= 1) {
        T o1 = __shfl_xor(m1, o), o2 = __shfl_xor(m2, o);
        int64_t osd = __shfl_xor(sd, o);
        top2_push(m1, m2, o1);
        top2_push(m1, m2, o2);
        sd += osd;
    }
    __shared__ double s1[4], s2[4];
    __shared__ int64_t ss[4];
    if (lane == 0) {
        s1[wave] = (double)m1;
        s2[wave] = (double)m2;
        ss[wave] = sd;
    }
    __syncthreads();
    if (tid == 0) {
        double a1 = s1[0], a2 = s2[0];
        int64_t t = ss[0];
        for (int w = 1; w < 4; ++w) {
            top2_push(a1, a2, s1[w]);
            top2_push(a1, a2, s2[w]);
            t += ss[w];
        }
        double *hp = slot_hpart(sa, slot);
        const size_t o = (size_t)k * kCols + c;
        hp[o] = a1;
        hp[kPushSplitMax * kCols + o] = a2;
        reinterpret_cast<int64_t *>(hp + 2 * kPushSplitMax * kCols)[o] = t;
    }
}

// Fused hop 2 for one column in LDS: the (w, 1/d(v)) contributions of the
// column are accumulated in a hash table in LDS (key w, unsigned fixed-point
// sum, 64-bit LDS atomics -- exact and order independent), then every table
// entry is converted once.  Used when the column's work sum_{v in N(u)} d(v)
// fits the table at half load; other columns take the global path.
constexpr int kHashCap = 12288;  // 144 KB of the 160 KB LDS

template <class T>
__global__ __launch_bounds__(512) void k_hop2_lds(QState qs, SlotArgs sa,
                                                  const int32_t *__restrict__ row_ptr,
                                                  const int32_t *__restrict__ col_idx,
                                                  const double *__restrict__ inv_deg_d, int shift)
{
    __shared__ int32_t s_key[kHashCap];
    __shared__ unsigned long long s_val[kHashCap];
    __shared__ int32_t s_pre[513];
    __shared__ int32_t s_v[512];
    __shared__ int32_t s_beg[512];
    __shared__ int32_t s_tmp[512];
    __shared__ double s1[8], s2[8];
    __shared__ int64_t ss[8];
    const int c = blockIdx.x;
    const int slot = blockIdx.y;
    const int j = c >> 1;
    const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
    const uint64_t *mask_p = sa.meta + 2 * sa.G + 4 * slot;  // per-column LDS-path mask
    const bool act = (mask_p[c >> 6] >> (c & 63)) & 1ull;
    T *out = slot_buf<T>(sa, slot, 1);
    uint32_t *out_bits = slot_bits(sa, slot, 1);
    T m1 = 0, m2 = 0;
    int64_t sd = 0;
    if (act) {
        for (int i = tid; i < kHashCap; i += 512) {
            s_key[i] = -1;
            s_val[i] = 0ull;
        }
        const int64_t q = qs.ord[slot_q0(sa, slot) + j];
        const int32_t u = (c & 1) ? qs.t[q] : qs.s[q];
        const int32_t b0 = row_ptr[u], du = row_ptr[u + 1] - b0;
        __syncthreads();
        for (int32_t base = 0; base < du; base += 512) {
            const int cnt = min(512, du - base);
            int32_t local = 0;
            for (int i = tid; i < min(cnt, tid + 1); ++i) {
                const int32_t v = col_idx[b0 + base + i];
                const int32_t rb = row_ptr[v];
                s_v[i] = v;
                s_beg[i] = rb;
                s_pre[i] = row_ptr[v + 1] - rb;
                local += s_pre[i];
            }
            s_tmp[tid] = local;
            __syncthreads();
            for (int o = 1; o < 512; o <<= 1) {
                int32_t add = tid >= o ? s_tmp[tid - o] : 0;
                __syncthreads();
                s_tmp[tid] += add;
                __syncthreads();
            }
            int32_t run = s_tmp[tid] - local;
            for (int i = tid; i < min(cnt, tid + 1); ++i) {
                const int32_t d = s_pre[i];
                s_pre[i] = run;
                run += d;
            }
            if (tid == 511) s_pre[cnt] = s_tmp[511];
            __syncthreads();
            const int32_t total = s_pre[cnt];
            for (int32_t p = tid; p < total; p += 512) {
                int lo = 0, hi = cnt;
                while (hi - lo > 1) {
                    const int mid = (lo + hi) >> 1;
                    if (s_pre[mid] <= p) lo = mid;
                    else hi = mid;
                }
                const int32_t v = s_v[lo];
                const int32_t w = col_idx[s_beg[lo] + (p - s_pre[lo])];
                // open addressing with linear probing; the table is never more
                // than half full (checked by the caller), so a slot is found
                uint32_t h = ((uint32_t)w * 2654435761u) % (uint32_t)kHashCap;
                for (;;) {
                    const int32_t k = s_key[h];
                    if (k == w) break;
                    if (k == -1) {
                        const int32_t old = atomicCAS(&s_key[h], -1, w);
                        if (old == -1 || old == w) break;
                    }
                    h = h + 1 == (uint32_t)kHashCap ? 0u : h + 1;
                }
                atomicAdd(&s_val[h], fixed_inv_deg(inv_deg_d[v], shift));
            }
            __syncthreads();
        }
        const uint32_t bit = 1u << (c & 31);
        for (int i = tid; i < kHashCap; i += 512) {
            const int32_t w = s_key[i];
            if (w < 0) continue;
            const T val = (T)(ldexp((double)s_val[i], -shift) * inv_deg_d[w]);
            out[(size_t)w * kCols + c] = val;
            atomicOr(out_bits + (size_t)w * kBitWords + (c >> 5), bit);
            top2_push(m1, m2, val);
            sd += row_ptr[w + 1] - row_ptr[w];
        }
    }
    if (!act) return;
    for (int o = 32; o > 0; o >>= 1) {
        T o1 = __shfl_xor(m1, o), o2 = __shfl_xor(m2, o);
        int64_t osd = __shfl_xor(sd, o);
        top2_push(m1, m2, o1);
        top2_push(m1, m2, o2);
        sd += osd;
    }
    if (lane == 0) {
        s1[wave] = (double)m1;
        s2[wave] = (double)m2;
        ss[wave] = sd;
    }
    __syncthreads();
    if (tid == 0) {
        double a1 = s1[0], a2 = s2[0];
        int64_t t = ss[0];
        for (int w = 1; w < 8; ++w) {
            top2_push(a1, a2, s1[w]);
            top2_push(a1, a2, s2[w]);
            t += ss[w];
        }
        // partial row 0 (the other rows of an LDS-path column stay zero)
        double *hp = slot_hpart(sa, slot);
        hp[c] = a1;
        hp[kPushSplitMax * kCols + c] = a2;
        reinterpret_cast<int64_t *>(hp + 2 * kPushSplitMax * kCols)[c] = t;
    }
}

geer_status launch_hop2_lds_group(geer_graph *g, const QueryCtx &c, const SlotArgs &sa,
                                  int nslots, int value_size, hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    const dim3 grid(kCols, nslots);
    int tok = prof_begin(g, st);
    if (value_size == 4)
        hipLaunchKernelGGL(k_hop2_lds<float>, grid, dim3(512), 0, st, c.qs, sa, g->d_row_ptr,
                           g->d_col_idx, g->d_inv_deg_d, g->fx_shift);
    else
        hipLaunchKernelGGL(k_hop2_lds<double>, grid, dim3(512), 0, st, c.qs, sa, g->d_row_ptr,
                           g->d_col_idx, g->d_inv_deg_d, g->fx_shift);
    prof_end(g, tok, PK_HOP2_LDS, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

int hop2_split(int ncols)
{
    // about 2048 blocks over the columns of the pass
    return std::max(kPushSplit, std::min(kPushSplitMax, 2048 / std::max(ncols, 1)));
}

geer_status launch_hop2_sparse(geer_graph *g, const QueryCtx &c, const SlotArgs &sa, int slot0,
                               int nslots, int value_size, int mode, int split, hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    if (split < 1 || split > kPushSplitMax) return fail(GEER_E_INVALID_ARG, "hop-2 split out of range");
    Workspace &ws = g->ws;
    // push and convert use accumulator block (slot - slot0) of each slot
    if (mode != 2 && nslots > ws.acc_slots)
        return fail(GEER_E_INVALID_ARG, "hop-2 push covers more slots than accumulators");
    unsigned long long *acc = ws.acc.as<unsigned long long>();
    const dim3 grid(kCols, split * nslots);
    int tok = prof_begin(g, st);
#define GEER_PUSH(T_, M_)                                                                      \
    hipLaunchKernelGGL((k_hop2_sparse<T_, M_>), grid, dim3(256), 0, st, c.qs, sa, slot0,        \
                       g->d_row_ptr, g->d_col_idx, g->d_inv_deg_d, acc, g->fx_shift, split)
    if (value_size == 4) {
        if (mode == 0) GEER_PUSH(float, 0);
        else if (mode == 1) GEER_PUSH(float, 1);
        else GEER_PUSH(float, 2);
    } else {
        if (mode == 0) GEER_PUSH(double, 0);
        else if (mode == 1) GEER_PUSH(double, 1);
        else GEER_PUSH(double, 2);
    }
#undef GEER_PUSH
    prof_end(g, tok, PK_HOP2_SPARSE, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

int ensure_hop2_acc(geer_graph *g, int want, hipStream_t st, geer_status *err)
{
    Workspace &ws = g->ws;
    *err = GEER_OK;
    if (ws.acc_slots >= want || (t_capturing && ws.acc_slots > 0)) return ws.acc_slots;
    // one block of n x kCols 64-bit accumulators per slot, within a quarter
    // of the free device memory (at least one block)
    const size_t per = (size_t)g->n * kCols * sizeof(unsigned long long);
    size_t free_b = 0, total_b = 0;
    if (hipMemGetInfo(&free_b, &total_b) != hipSuccess) free_b = 0;
    const size_t fit = (free_b + ws.acc.bytes) / 4 / per;
    const int slots = (int)std::max<size_t>(1, std::min<size_t>((size_t)want, fit));
    if (slots <= ws.acc_slots) return ws.acc_slots;
    ws.acc_slots = 0;  // reserve() releases the old blocks
    if ((*err = ws.acc.reserve((size_t)slots * per)) != GEER_OK) return 0;
    if ((*err = launch_zero(g, ws.acc.ptr, (size_t)slots * per, st)) != GEER_OK) return 0;
    ws.acc_slots = slots;
    return slots;
}

geer_status launch_colstat_group(geer_graph *g, const SlotArgs &sa, int nslots, int split,
                                 hipStream_t st)
{
    if (nslots <= 0) return GEER_OK;
    int tok = prof_begin(g, st);
    hipLaunchKernelGGL(k_colstat_group, dim3(kCols, nslots), dim3(64), 0, st, sa, split);
    prof_end(g, tok, PK_COLSTAT, 0.0, 0.0, st);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

// Fill a buffer with zeros (a kernel, so it can live inside captured graphs).
__global__ void k_zero_words(uint4 *__restrict__ p, size_t n16)
{
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n16;
         i += (size_t)gridDim.x * blockDim.x)
        p[i] = make_uint4(0, 0, 0, 0);
}

geer_status launch_zero(geer_graph *g, void *p, size_t bytes, hipStream_t st)
{
    if (bytes % 16 != 0) return fail(GEER_E_INVALID_ARG, "zero fill needs 16-byte multiples");
    const size_t n16 = bytes / 16;
    const int blocks = (int)std::min<size_t>((n16 + 255) / 256, (size_t)g->num_cus * 16);
    hipLaunchKernelGGL(k_zero_words, dim3(std::max(blocks, 1)), dim3(256), 0, st, (uint4 *)p, n16);
    GEER_HIP(hipGetLastError());
    return GEER_OK;
}

}  // namespace geer
