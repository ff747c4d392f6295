/*
 * CPU FP64 checker for the GEER estimator of pairwise effective resistance
 * (Yang & Tang, "Efficient Estimation of Pairwise Effective Resistance").
 *
 * TEST INFRASTRUCTURE ONLY.  This file is the slow, plain reference that the
 * GPU library is checked against.  It shares no code with the GPU library and
 * must only be called from the test-suite, the smoke check and the
 * benchmark's CPU-baseline leg.  Nothing in the product path may load it.
 *
 * Every function follows one passage of the paper, cited by section and
 * equation/algorithm.  Arithmetic is FP64 throughout; loops run in the
 * natural order (no blocking, fusion or reordering).
 *
 * Readings of passages the paper leaves open (all documented alongside the
 * GPU design as well):
 *   - P = D^-1 A is row-stochastic, so (P x)(v) = (1/d(v)) sum_{u in N(v)} x(u)
 *     and after i products x = P^i e_s holds x(v) = p_i(v, s)  (Section 4.1.1,
 *     the identity for the SMM vectors).
 *   - max_k(x) is the k-th entry of x sorted descending, counting repeated
 *     values (notation table; needed for the walk-sum bound of Lemma 3.3).
 *   - A walk of length l_f visits w_1..w_{l_f}; the start node w_0 is not
 *     part of the sum in Z_k (Section 3.3.1 and the proof of the walk-sum lemma).
 *   - Batches draw fresh walks (Section 3.2.1: results of a failed batch are
 *     discarded).  eta_1 = ceil(eta_star / 2^(tau-1)); after batch tau the loop ends.
 *   - The empirical variance is clamped at zero against rounding.
 *   - l = max(0, ceil(...)) in Eq. (ell); s == t returns 0 without work.
 *   - The greedy switch (Eq. smm-amc) uses the structural supports of the
 *     current SMM vectors (nodes reached by a walk of exactly l_b steps) and
 *     h(l - l_b) = (2^tau - 1) * eta_1 computed from the current vectors.
 *   - The paper names no random generator.  Walks use Philox4x32-10 (Salmon,
 *     Moraes, Dror, Shaw, SC'11) with counter (step>>2, k, (batch<<1)|side, q)
 *     and key (seed_lo, seed_hi); the draw is output word (step & 3) and the
 *     next node is row u's (draw mod d(u))-th CSR entry.
 */

#include <math.h>
#include <pthread.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

/* ------------------------------------------------------------------------ */
/* Philox4x32-10 counter-based generator (Salmon et al., SC'11, Section 3).  */
/* Round function: two 32x32->64 multiplications by fixed odd constants,    */
/* the high halves xor-ed with the other words and the round key; the key   */
/* advances by the Weyl constants (golden ratio, sqrt(3)-1) between rounds. */
/* ------------------------------------------------------------------------ */

void oracle_philox4x32_10(const uint32_t ctr[4], const uint32_t key[2], uint32_t out[4])
{
    uint32_t x0 = ctr[0], x1 = ctr[1], x2 = ctr[2], x3 = ctr[3];
    uint32_t k0 = key[0], k1 = key[1];
    for (int round = 0; round < 10; ++round) {
        uint64_t p0 = (uint64_t)0xD2511F53u * (uint64_t)x0;
        uint64_t p1 = (uint64_t)0xCD9E8D57u * (uint64_t)x2;
        uint32_t hi0 = (uint32_t)(p0 >> 32), lo0 = (uint32_t)p0;
        uint32_t hi1 = (uint32_t)(p1 >> 32), lo1 = (uint32_t)p1;
        uint32_t y0 = hi1 ^ x1 ^ k0;
        uint32_t y1 = lo1;
        uint32_t y2 = hi0 ^ x3 ^ k1;
        uint32_t y3 = lo0;
        x0 = y0; x1 = y1; x2 = y2; x3 = y3;
        k0 += 0x9E3779B9u;
        k1 += 0xBB67AE85u;
    }
    out[0] = x0; out[1] = x1; out[2] = x2; out[3] = x3;
}

/* One 32-bit draw of the walk sampler. */
static uint32_t walk_draw(uint64_t seed, uint32_t q, uint32_t batch, uint32_t k,
                          uint32_t side, uint32_t step)
{
    uint32_t ctr[4] = { step >> 2, k, (batch << 1) | side, q };
    uint32_t key[2] = { (uint32_t)seed, (uint32_t)(seed >> 32) };
    uint32_t out[4];
    oracle_philox4x32_10(ctr, key, out);
    return out[step & 3u];
}

/* ------------------------------------------------------------------------ */
/* Graph helpers                                                             */
/* ------------------------------------------------------------------------ */

static inline int64_t deg_of(const int64_t *rp, int64_t v) { return rp[v + 1] - rp[v]; }

/* One product with the transition matrix: y = P x, (P x)(v) = mean of x over N(v).
 * Section 4.1.1 (Algorithm SMM, the update of s* and t*). */
void oracle_smm_hop(int64_t n, const int64_t *rp, const int32_t *ci,
                    const double *x, double *y)
{
    for (int64_t v = 0; v < n; ++v) {
        double acc = 0.0;
        for (int64_t e = rp[v]; e < rp[v + 1]; ++e) acc += x[ci[e]];
        y[v] = acc / (double)deg_of(rp, v);
    }
}

/* Structural support after one more product: v is reached iff a neighbour was. */
static void support_hop(int64_t n, const int64_t *rp, const int32_t *ci,
                        const unsigned char *sx, unsigned char *sy)
{
    for (int64_t v = 0; v < n; ++v) {
        unsigned char any = 0;
        for (int64_t e = rp[v]; e < rp[v + 1] && !any; ++e) any = sx[ci[e]];
        sy[v] = any;
    }
}

static int64_t support_degree_sum(int64_t n, const int64_t *rp, const unsigned char *sx)
{
    int64_t total = 0;
    for (int64_t v = 0; v < n; ++v) if (sx[v]) total += deg_of(rp, v);
    return total;
}

/* Largest and second-largest entries, counting repeats (notation table). */
void oracle_top2(int64_t n, const double *x, double *max1, double *max2)
{
    double m1 = -INFINITY, m2 = -INFINITY;
    for (int64_t v = 0; v < n; ++v) {
        if (x[v] > m1) { m2 = m1; m1 = x[v]; }
        else if (x[v] > m2) { m2 = x[v]; }
    }
    *max1 = m1;
    *max2 = m2;
}

/* ------------------------------------------------------------------------ */
/* Scalar formulas                                                           */
/* ------------------------------------------------------------------------ */

/* Eq. (ell), Theorem 3.1: per-pair maximum walk length, clamped at 0. */
int32_t oracle_ell(double ds, double dt, double eps, double lambda)
{
    if (!(lambda > 0.0)) return 0;
    double v = log((2.0 / ds + 2.0 / dt) / (eps * (1.0 - lambda))) / log(1.0 / lambda) - 1.0;
    double c = ceil(v);
    if (c < 0.0) return 0;
    return (int32_t)c;
}

/* Eq. (old-ell): the maximum length of Peng et al., kept for comparison. */
int32_t oracle_ell_peng(double eps, double lambda)
{
    if (!(lambda > 0.0)) return 0;
    double v = log(4.0 / (eps - eps * lambda)) / log(1.0 / lambda) - 1.0;
    double c = ceil(v);
    if (c < 0.0) return 0;
    return (int32_t)c;
}

/* Eq. (Delta-st): psi from the top-2 entries of the two input vectors. */
double oracle_psi(int32_t lf, double m1s, double m2s, double m1t, double m2t, double ds, double dt)
{
    double up = (double)((lf + 1) / 2);
    double dn = (double)(lf / 2);
    return 2.0 * up * (m1s / ds + m1t / dt) + 2.0 * dn * (m2s / ds + m2t / dt);
}

/* Eq. (etas-star): Hoeffding cap on the walk-pair count. */
double oracle_eta_star(double psi, double eps, int32_t tau, double delta)
{
    return 2.0 * psi * psi * log(2.0 * (double)tau / delta) / (eps * eps);
}

/* Algorithm AMC, initial batch size: ceil(eta* / 2^(tau-1)). */
uint64_t oracle_eta1(double eta_star, int32_t tau)
{
    double v = ceil(eta_star / ldexp(1.0, tau - 1));
    if (v <= 0.0) return 0;
    return (uint64_t)v;
}

/* Section 3.3.2: total walk pairs over tau batches, h = (2^tau - 1) eta_1. */
double oracle_h(double eta_star, int32_t tau)
{
    return (ldexp(1.0, tau) - 1.0) * (double)oracle_eta1(eta_star, tau);
}

/* Eq. (fx), empirical Bernstein half-width. */
double oracle_bernstein(double nz, double var, double psi, double delta)
{
    double lg = log(3.0 / delta);
    return sqrt(2.0 * var * lg / nz) + 3.0 * psi * lg / nz;
}

/* ------------------------------------------------------------------------ */
/* Random walks                                                              */
/* ------------------------------------------------------------------------ */

/* Record the nodes w_1..w_lf of one walk (Algorithm AMC, walks S_k / T_k). */
void oracle_walk_trace(const int64_t *rp, const int32_t *ci, int32_t start, int32_t lf,
                       uint64_t seed, uint32_t q, uint32_t batch, uint32_t k, uint32_t side,
                       int32_t *trace)
{
    int64_t u = start;
    for (int32_t step = 0; step < lf; ++step) {
        uint32_t r = walk_draw(seed, q, batch, k, side, (uint32_t)step);
        int64_t d = deg_of(rp, u);
        u = ci[rp[u] + (int64_t)(r % (uint32_t)d)];
        trace[step] = (int32_t)u;
    }
}

/* Sum of the weight function over the visited nodes of one walk. */
static double walk_sum(const int64_t *rp, const int32_t *ci, int32_t start, int32_t lf,
                       uint64_t seed, uint32_t q, uint32_t batch, uint32_t k, uint32_t side,
                       const double *x, const double *y, double ds, double dt)
{
    double acc = 0.0;
    int64_t u = start;
    for (int32_t step = 0; step < lf; ++step) {
        uint32_t r = walk_draw(seed, q, batch, k, side, (uint32_t)step);
        int64_t d = deg_of(rp, u);
        u = ci[rp[u] + (int64_t)(r % (uint32_t)d)];
        if (side == 0) acc += x[u] / ds - y[u] / dt;   /* walk S_k from s */
        else           acc += y[u] / dt - x[u] / ds;   /* walk T_k from t */
    }
    return acc;
}

/* Per-query record shared with the Python wrapper (layout mirrored there). */
typedef struct {
    int32_t ell, ell_b, lf, batches_run;
    int64_t eta1, walk_pairs, supp_sum;
    double r_b, r_f, r, psi, eta_star, z_sum, z2_sum, var, f_last;
} oracle_stats;

/* Algorithm AMC (Section 3.2.2) with arbitrary non-negative input vectors.
 * Returns r_f; fills the AMC fields of *st. */
double oracle_amc(const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                  const double *x, const double *y, int64_t n, double eps, int32_t lf,
                  int32_t tau, double delta, uint64_t seed, uint32_t q, oracle_stats *st)
{
    double ds = (double)deg_of(rp, s), dt = (double)deg_of(rp, t);
    st->lf = lf;
    st->batches_run = 0;
    st->walk_pairs = 0;
    st->eta1 = 0;
    st->psi = 0.0;
    st->eta_star = 0.0;
    st->z_sum = st->z2_sum = st->var = st->f_last = 0.0;
    if (lf <= 0) return 0.0;
    double m1s, m2s, m1t, m2t;
    oracle_top2(n, x, &m1s, &m2s);
    oracle_top2(n, y, &m1t, &m2t);
    double psi = oracle_psi(lf, m1s, m2s, m1t, m2t, ds, dt);
    double eta_star = oracle_eta_star(psi, eps, tau, delta);
    uint64_t eta = oracle_eta1(eta_star, tau);
    st->psi = psi;
    st->eta_star = eta_star;
    st->eta1 = (int64_t)eta;
    if (eta == 0) return 0.0;
    double z = 0.0;
    for (int32_t i = 0; i < tau; ++i) {
        double zs = 0.0, z2 = 0.0;
        for (uint64_t k = 0; k < eta; ++k) {
            double zk = walk_sum(rp, ci, s, lf, seed, q, (uint32_t)i, (uint32_t)k, 0, x, y, ds, dt)
                      + walk_sum(rp, ci, t, lf, seed, q, (uint32_t)i, (uint32_t)k, 1, x, y, ds, dt);
            zs += zk;
            z2 += zk * zk;
        }
        z = zs / (double)eta;
        double var = z2 / (double)eta - z * z;
        if (var < 0.0) var = 0.0;
        double f = oracle_bernstein((double)eta, var, psi, delta / (double)tau);
        st->batches_run = i + 1;
        st->walk_pairs += (int64_t)eta;
        st->z_sum = zs;
        st->z2_sum = z2;
        st->var = var;
        st->f_last = f;
        if (f <= eps / 2.0) break;
        if (i + 1 < tau) eta *= 2;
    }
    return z;
}

/* The 4-term hop increment of r_b (Algorithm SMM / GEER). */
static double rb_term(const double *x, const double *y, int32_t s, int32_t t, double ds, double dt)
{
    return x[s] / ds + y[t] / dt - x[t] / ds - y[s] / dt;
}

/* Scratch owned by one worker thread. */
typedef struct { double *x, *y, *x2, *y2; unsigned char *sx, *sy, *sx2, *sy2; } work_buf;

static int work_alloc(work_buf *w, int64_t n)
{
    w->x = calloc((size_t)n, sizeof(double));
    w->y = calloc((size_t)n, sizeof(double));
    w->x2 = calloc((size_t)n, sizeof(double));
    w->y2 = calloc((size_t)n, sizeof(double));
    w->sx = calloc((size_t)n, 1);
    w->sy = calloc((size_t)n, 1);
    w->sx2 = calloc((size_t)n, 1);
    w->sy2 = calloc((size_t)n, 1);
    return (w->x && w->y && w->x2 && w->y2 && w->sx && w->sy && w->sx2 && w->sy2) ? 0 : -1;
}

static void work_free(work_buf *w)
{
    free(w->x); free(w->y); free(w->x2); free(w->y2);
    free(w->sx); free(w->sy); free(w->sx2); free(w->sy2);
}

/* Algorithm GEER (Section 4.2) for one pair.
 * schedule 0: greedy switch of Eq. (smm-amc);  schedule 1: exactly
 * min(fixed_lb, l) SMM iterations.  Returns r'(s, t). */
static double geer_one(int64_t n, const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                       double eps, double lambda, int32_t tau, double delta, uint64_t seed,
                       uint32_t q, int32_t schedule, int32_t fixed_lb, int32_t ell_rule,
                       work_buf *w, oracle_stats *st)
{
    memset(st, 0, sizeof(*st));
    if (s == t) return 0.0;                              /* r(s,s) = 0, Section 2.2 */
    double ds = (double)deg_of(rp, s), dt = (double)deg_of(rp, t);
    /* Eq. (ell), or Eq. (old-ell) for the comparison variant of Section 3.1 */
    int32_t ell = ell_rule == 1 ? oracle_ell_peng(eps, lambda) : oracle_ell(ds, dt, eps, lambda);
    st->ell = ell;
    double *x = w->x, *y = w->y, *x2 = w->x2, *y2 = w->y2;
    unsigned char *sx = w->sx, *sy = w->sy, *sx2 = w->sx2, *sy2 = w->sy2;
    memset(x, 0, (size_t)n * sizeof(double));
    memset(y, 0, (size_t)n * sizeof(double));
    memset(sx, 0, (size_t)n);
    memset(sy, 0, (size_t)n);
    x[s] = 1.0; y[t] = 1.0; sx[s] = 1; sy[t] = 1;
    double rb = rb_term(x, y, s, t, ds, dt);
    int32_t lb = 0;
    int32_t target = schedule == 1 ? (fixed_lb < ell ? fixed_lb : ell) : ell;
    if (target < 0) target = 0;
    int64_t supp_sum = support_degree_sum(n, rp, sx) + support_degree_sum(n, rp, sy);
    if (ell > 0 && target > 0) {
        for (;;) {
            oracle_smm_hop(n, rp, ci, x, x2);
            oracle_smm_hop(n, rp, ci, y, y2);
            support_hop(n, rp, ci, sx, sx2);
            support_hop(n, rp, ci, sy, sy2);
            double *td = x; x = x2; x2 = td;
            td = y; y = y2; y2 = td;
            unsigned char *tb = sx; sx = sx2; sx2 = tb;
            tb = sy; sy = sy2; sy2 = tb;
            rb += rb_term(x, y, s, t, ds, dt);
            lb += 1;
            supp_sum = support_degree_sum(n, rp, sx) + support_degree_sum(n, rp, sy);
            if (lb >= target) break;
            if (schedule == 0) {
                double m1s, m2s, m1t, m2t;
                oracle_top2(n, x, &m1s, &m2s);
                oracle_top2(n, y, &m1t, &m2t);
                double psi = oracle_psi(ell - lb, m1s, m2s, m1t, m2t, ds, dt);
                double h = oracle_h(oracle_eta_star(psi, eps, tau, delta), tau);
                if ((double)supp_sum > h) break;
            }
        }
    }
    st->ell_b = lb;
    st->r_b = rb;
    st->supp_sum = supp_sum;
    double rf = oracle_amc(rp, ci, s, t, x, y, n, eps, ell - lb, tau, delta, seed, q, st);
    st->r_f = rf;
    st->r = rb + rf;
    return rb + rf;
}

/* Truncated series r_l (Eq. r-ell): l products with P, nothing sampled. */
static double series_one(int64_t n, const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                         int32_t ell, work_buf *w)
{
    if (s == t) return 0.0;
    double ds = (double)deg_of(rp, s), dt = (double)deg_of(rp, t);
    double *x = w->x, *y = w->y, *x2 = w->x2, *y2 = w->y2;
    memset(x, 0, (size_t)n * sizeof(double));
    memset(y, 0, (size_t)n * sizeof(double));
    x[s] = 1.0; y[t] = 1.0;
    double r = rb_term(x, y, s, t, ds, dt);
    for (int32_t i = 1; i <= ell; ++i) {
        oracle_smm_hop(n, rp, ci, x, x2);
        oracle_smm_hop(n, rp, ci, y, y2);
        double *td = x; x = x2; x2 = td;
        td = y; y = y2; y2 = td;
        r += rb_term(x, y, s, t, ds, dt);
    }
    return r;
}

/* Jacobi-preconditioned conjugate gradients on L z = e_s - e_t (Definition 2.1):
 * r(s,t) = (e_s - e_t)^T z.  L is singular with null space span(1); the
 * right-hand side is orthogonal to it, so CG stays in the range. */
static double cg_one(int64_t n, const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                     double tol, int32_t max_iter, work_buf *w, int32_t *iters_out)
{
    if (s == t) { *iters_out = 0; return 0.0; }
    double *z = w->x, *r = w->y, *p = w->x2, *ap = w->y2;
    memset(z, 0, (size_t)n * sizeof(double));
    memset(r, 0, (size_t)n * sizeof(double));
    r[s] = 1.0; r[t] = -1.0;
    double bnorm = sqrt(2.0);
    double rz = 0.0;
    for (int64_t v = 0; v < n; ++v) { p[v] = r[v] / (double)deg_of(rp, v); rz += r[v] * p[v]; }
    int32_t it = 0;
    for (; it < max_iter; ++it) {
        double pap = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            double acc = (double)deg_of(rp, v) * p[v];
            for (int64_t e = rp[v]; e < rp[v + 1]; ++e) acc -= p[ci[e]];
            ap[v] = acc;
            pap += p[v] * acc;
        }
        double alpha = rz / pap;
        double rr = 0.0;
        for (int64_t v = 0; v < n; ++v) {
            z[v] += alpha * p[v];
            r[v] -= alpha * ap[v];
            rr += r[v] * r[v];
        }
        if (sqrt(rr) <= tol * bnorm) { ++it; break; }
        double rz_new = 0.0;
        for (int64_t v = 0; v < n; ++v) rz_new += r[v] * r[v] / (double)deg_of(rp, v);
        double beta = rz_new / rz;
        rz = rz_new;
        for (int64_t v = 0; v < n; ++v) p[v] = r[v] / (double)deg_of(rp, v) + beta * p[v];
    }
    *iters_out = it;
    return z[s] - z[t];
}

/* ------------------------------------------------------------------------ */
/* Multi-query drivers (threads over queries; each query is independent).    */
/* ------------------------------------------------------------------------ */

typedef struct {
    int kind; /* 0 geer, 1 series, 2 cg */
    int64_t n, nq;
    const int64_t *rp;
    const int32_t *ci;
    const int32_t *s, *t;
    const double *eps;
    double lambda, delta, tol;
    int32_t tau, schedule, max_iter;
    const int32_t *fixed_lb;   /* per query, schedule 1 */
    const int32_t *tau_arr;    /* per query batch count, or NULL for `tau` */
    int32_t ell_rule;          /* 0: Eq. (ell), 1: Eq. (old-ell) */
    const int32_t *ell_in;     /* per query, series */
    uint64_t seed;
    const int64_t *qid;        /* global query index for the walk counter, or NULL */
    double *r_out;
    oracle_stats *stats;
    int32_t *iters;
    int64_t next;
    pthread_mutex_t lock;
    int failed;
} job_t;

static void *worker(void *arg)
{
    job_t *j = (job_t *)arg;
    work_buf w;
    if (work_alloc(&w, j->n) != 0) {
        pthread_mutex_lock(&j->lock);
        j->failed = 1;
        pthread_mutex_unlock(&j->lock);
        work_free(&w);
        return NULL;
    }
    for (;;) {
        pthread_mutex_lock(&j->lock);
        int64_t i = j->next++;
        pthread_mutex_unlock(&j->lock);
        if (i >= j->nq) break;
        if (j->kind == 0) {
            oracle_stats st;
            uint32_t q = (uint32_t)(j->qid ? j->qid[i] : i);
            int32_t flb = j->fixed_lb ? j->fixed_lb[i] : 0;
            int32_t tq = j->tau_arr ? j->tau_arr[i] : j->tau;
            j->r_out[i] = geer_one(j->n, j->rp, j->ci, j->s[i], j->t[i], j->eps[i], j->lambda,
                                   tq, j->delta, j->seed, q, j->schedule, flb, j->ell_rule, &w,
                                   &st);
            if (j->stats) j->stats[i] = st;
        } else if (j->kind == 1) {
            j->r_out[i] = series_one(j->n, j->rp, j->ci, j->s[i], j->t[i], j->ell_in[i], &w);
        } else {
            int32_t its = 0;
            j->r_out[i] = cg_one(j->n, j->rp, j->ci, j->s[i], j->t[i], j->tol, j->max_iter, &w, &its);
            if (j->iters) j->iters[i] = its;
        }
    }
    work_free(&w);
    return NULL;
}

static int run_job(job_t *j, int32_t threads)
{
    if (threads < 1) threads = 1;
    if (threads > 256) threads = 256;
    pthread_t tid[256];
    j->next = 0;
    j->failed = 0;
    pthread_mutex_init(&j->lock, NULL);
    int32_t started = 0;
    for (int32_t i = 0; i < threads; ++i) {
        if (pthread_create(&tid[i], NULL, worker, j) != 0) break;
        ++started;
    }
    if (started == 0) worker(j);
    for (int32_t i = 0; i < started; ++i) pthread_join(tid[i], NULL);
    pthread_mutex_destroy(&j->lock);
    return j->failed ? -1 : 0;
}

/* GEER for a batch of pairs (Algorithm GEER).  Returns 0 on success. */
int oracle_geer(int64_t n, const int64_t *rp, const int32_t *ci, int64_t nq,
                const int32_t *s, const int32_t *t, const double *eps, double lambda,
                int32_t tau, double delta, uint64_t seed, int32_t schedule,
                const int32_t *fixed_lb, const int64_t *qid, int32_t threads,
                double *r_out, oracle_stats *stats, const int32_t *tau_arr, int32_t ell_rule)
{
    job_t j;
    memset(&j, 0, sizeof(j));
    j.tau_arr = tau_arr;
    j.ell_rule = ell_rule;
    j.kind = 0; j.n = n; j.nq = nq; j.rp = rp; j.ci = ci; j.s = s; j.t = t; j.eps = eps;
    j.lambda = lambda; j.tau = tau; j.delta = delta; j.seed = seed; j.schedule = schedule;
    j.fixed_lb = fixed_lb; j.qid = qid; j.r_out = r_out; j.stats = stats;
    return run_job(&j, threads);
}

/* Truncated series r_l for given per-pair l (Eq. r-ell). */
int oracle_series(int64_t n, const int64_t *rp, const int32_t *ci, int64_t nq,
                  const int32_t *s, const int32_t *t, const int32_t *ell, int32_t threads,
                  double *r_out)
{
    job_t j;
    memset(&j, 0, sizeof(j));
    j.kind = 1; j.n = n; j.nq = nq; j.rp = rp; j.ci = ci; j.s = s; j.t = t; j.ell_in = ell;
    j.r_out = r_out;
    return run_job(&j, threads);
}

/* Exact r(s,t) by PCG (Definition 2.1). */
int oracle_exact_cg(int64_t n, const int64_t *rp, const int32_t *ci, int64_t nq,
                    const int32_t *s, const int32_t *t, double tol, int32_t max_iter,
                    int32_t threads, double *r_out, int32_t *iters)
{
    job_t j;
    memset(&j, 0, sizeof(j));
    j.kind = 2; j.n = n; j.nq = nq; j.rp = rp; j.ci = ci; j.s = s; j.t = t; j.tol = tol;
    j.max_iter = max_iter; j.r_out = r_out; j.iters = iters;
    return run_job(&j, threads);
}

/* SMM vectors after exactly `hops` products, with structural supports and
 * r_b (Algorithm SMM).  x_out, y_out: n doubles each; supp_out: 2n bytes. */
void oracle_smm_vectors(int64_t n, const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                        int32_t hops, double *x_out, double *y_out, unsigned char *supp_out,
                        double *rb_out)
{
    work_buf w;
    if (work_alloc(&w, n) != 0) { work_free(&w); *rb_out = NAN; return; }
    double ds = (double)deg_of(rp, s), dt = (double)deg_of(rp, t);
    double *x = w.x, *y = w.y, *x2 = w.x2, *y2 = w.y2;
    unsigned char *sx = w.sx, *sy = w.sy, *sx2 = w.sx2, *sy2 = w.sy2;
    x[s] = 1.0; y[t] = 1.0; sx[s] = 1; sy[t] = 1;
    double rb = rb_term(x, y, s, t, ds, dt);
    for (int32_t i = 0; i < hops; ++i) {
        oracle_smm_hop(n, rp, ci, x, x2);
        oracle_smm_hop(n, rp, ci, y, y2);
        support_hop(n, rp, ci, sx, sx2);
        support_hop(n, rp, ci, sy, sy2);
        double *td = x; x = x2; x2 = td;
        td = y; y = y2; y2 = td;
        unsigned char *tb = sx; sx = sx2; sx2 = tb;
        tb = sy; sy = sy2; sy2 = tb;
        rb += rb_term(x, y, s, t, ds, dt);
    }
    memcpy(x_out, x, (size_t)n * sizeof(double));
    memcpy(y_out, y, (size_t)n * sizeof(double));
    memcpy(supp_out, sx, (size_t)n);
    memcpy(supp_out + n, sy, (size_t)n);
    *rb_out = s == t ? 0.0 : rb;
    work_free(&w);
}

/* All Z_k samples of one AMC batch, for statistical tests (Eq. x-exp). */
void oracle_amc_samples(const int64_t *rp, const int32_t *ci, int32_t s, int32_t t,
                        const double *x, const double *y, int32_t lf, uint64_t seed,
                        uint32_t q, uint32_t batch, int64_t count, double *z_out)
{
    double ds = (double)deg_of(rp, s), dt = (double)deg_of(rp, t);
    for (int64_t k = 0; k < count; ++k)
        z_out[k] = walk_sum(rp, ci, s, lf, seed, q, batch, (uint32_t)k, 0, x, y, ds, dt)
                 + walk_sum(rp, ci, t, lf, seed, q, batch, (uint32_t)k, 1, x, y, ds, dt);
}

int oracle_stats_size(void) { return (int)sizeof(oracle_stats); }
