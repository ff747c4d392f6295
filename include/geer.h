/*
 * geer.h -- C ABI of the MI355X GEER library.
 *
 * GEER answers epsilon-approximate pairwise effective resistance queries
 * (Yang & Tang, "Efficient Estimation of Pairwise Effective Resistance",
 * Definition 2.2): given an undirected, unweighted, connected, non-bipartite
 * graph G and pairs (s, t) with additive error eps, it returns r'(s,t) with
 * |r'(s,t) - r(s,t)| <= eps with probability at least 1 - delta.
 *
 * The computation is Algorithm 3 (GEER): a per-pair maximum walk length l
 * (Eq. ell, Theorem 3.1), l_b products with the transition matrix
 * P = D^-1 A (Algorithm 2, SMM), then adaptive Monte Carlo walks from the SMM
 * frontier (Algorithm 1, AMC) with the empirical-Bernstein stop rule
 * (Lemma 3.2, Eq. fx) and the Hoeffding cap eta* (Eq. etas-star).
 *
 * Conventions for every entry point:
 *   - All functions return GEER_OK (0) or a negative geer_status.  On error
 *     nothing has been written to any output, and geer_last_error() returns a
 *     thread-local message describing the failure.
 *   - Host pointers are owned by the caller and are not retained after the
 *     call returns.  Device pointers (the *_device variants) must be HIP
 *     device allocations on the graph's device; the caller owns them.
 *   - A geer_graph may be used by one host thread / one stream at a time.
 *   - Node ids are 0-based int32.  The graph must be given in canonical CSR
 *     form: symmetric, no self-loops, no duplicate entries, every degree >= 1,
 *     each row sorted ascending.  The order of a row is part of the walk
 *     definition (the next node of a walk at u is row u's
 *     (draw mod d(u))-th entry).
 *
 * Walk randomness (the paper names no generator): Philox4x32-10 (Salmon,
 * Moraes, Dror, Shaw, SC'11) with key (seed low word, seed high word) and
 * counter (step >> 2, k, (batch << 1) | side, q).  step counts from 0 within
 * a walk, k is the walk-pair index within AMC batch `batch` (0-based), side
 * is 0 for the walk from s and 1 for the walk from t, and q is the query's
 * index (its position in the call plus geer_params.qid_offset).  The draw of a
 * step is output word (step & 3).  Walk node sequences are therefore integer
 * exact and reproducible on any implementation of this specification.
 */
#ifndef GEER_H
#define GEER_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
    GEER_OK = 0,
    GEER_E_INVALID_ARG = -1,   /* bad size, pointer, eps, delta, tau, node id, ... */
    GEER_E_GRAPH = -2,         /* CSR not canonical: asymmetric, self-loop, duplicate,
                                  unsorted row, degree 0, bad offsets */
    GEER_E_NOT_CONNECTED = -3, /* graph has more than one connected component */
    GEER_E_BIPARTITE = -4,     /* lambda >= 1 (bipartite graph, Theorem 3.1 needs lambda < 1) */
    GEER_E_NO_LAMBDA = -5,     /* query issued before lambda was set or computed */
    GEER_E_OOM = -6,           /* device allocation failed or scratch cap exceeded */
    GEER_E_DEVICE = -7,        /* a HIP runtime call failed */
    GEER_E_MODEL = -8          /* learned-scheduler model missing, malformed or unusable */
} geer_status;

/* Opaque handles. */
typedef struct geer_graph geer_graph;  /* device copy of the CSR + per-graph scratch */
typedef struct geer_model geer_model;  /* learned-scheduler weights (host + device copies) */

/* SMM depth schedule. */
enum {
    GEER_SCHEDULE_GREEDY = 0,  /* the paper's switch rule, Eq. (smm-amc) */
    GEER_SCHEDULE_LEARNED = 1, /* l_b and tau from a geer_model; greedy is the fallback */
    GEER_SCHEDULE_FIXED = 2    /* l_b = min(fixed_ell_b[q], l) for every query */
};

/* geer_params.flags */
enum {
    GEER_FLAG_FP64_VECTORS = 1u << 0, /* keep SMM vectors in FP64 instead of FP32 */
    GEER_FLAG_GRAPH_LAUNCH = 1u << 1, /* FIXED / LEARNED: after the depths are known (one
                                         read of them), run the SMM and AMC launches of every
                                         group of known depth as one captured hipGraph, and
                                         replay that graph on a later call that derives the
                                         same launches (same pairs, depths, batch counts and
                                         buffers).  Results are bit-identical to the direct
                                         launches.  Groups of the greedy switch (the GREEDY
                                         schedule, LEARNED pairs that fall back) decide at
                                         every hop from the vectors and are launched directly
                                         after the graph.  The captured AMC rounds keep their
                                         chunk partials in a reserved 256 MB buffer: a round
                                         needing more (over 5.4e8 walk pairs in one group)
                                         makes the call return GEER_E_OOM */
    GEER_FLAG_PENG_ELL = 1u << 2 /* l by Eq. (old-ell) (Peng et al.'s length, Section 3.1) for every
                                    pair instead of Eq. (ell): the paper's comparison variant */
};

typedef struct geer_params {
    double delta;                /* failure probability, 0 < delta < 1 (default 0.01) */
    int32_t tau;                 /* number of AMC batches, 1..30 (default 5) */
    int32_t schedule;            /* GEER_SCHEDULE_* (default GREEDY) */
    uint64_t seed;               /* Philox key (default 0) */
    int64_t qid_offset;          /* added to a query's position to form its walk counter id */
    const int32_t *fixed_ell_b;  /* FIXED: host array [nq] of requested SMM depths (>= 0) */
    const geer_model *model;     /* LEARNED: the scheduler */
    void *stream;                /* hipStream_t to run on, or NULL for the library's stream */
    int32_t batch_queries;       /* queries per SMM batch, 1..64 (0 = 64) */
    int32_t col_tile;            /* dense SpMM column tile 32/64/128 (0 = autotuned per hop) */
    int32_t walk_ilp;            /* 0 or 1: one walk per lane (the walk kernel is bound by random
                                    line fetches, which interleaving more walks per lane does not
                                    raise); other values are rejected */
    int32_t group_batches;       /* batches per group: their SMM runs, then one AMC phase for all
                                    of them (0 = auto, at most 32).  With more than one group, two
                                    slot sets alternate and a group's AMC phase overlaps the next
                                    group's SMM on a second library stream */
    uint32_t flags;              /* GEER_FLAG_* */
    int32_t reserved[7];
} geer_params;

/* Per-query record (optional output of geer_query). */
typedef struct geer_query_stats {
    int32_t ell;          /* Eq. (ell), or Eq. (old-ell) with GEER_FLAG_PENG_ELL */
    int32_t ell_b;        /* SMM products performed */
    int32_t tau;          /* AMC batches allowed */
    int32_t batches_run;  /* AMC batches performed */
    int32_t stop_reason;  /* GEER_STOP_* */
    int32_t fallback;     /* LEARNED: 1 if the greedy schedule was used instead */
    int64_t eta1;         /* first AMC batch size (walk pairs) */
    int64_t walk_pairs;   /* total walk pairs sampled */
    int64_t supp_sum;     /* sum of degrees over the supports of the final SMM vectors */
    double r_b;           /* deterministic part (hops 0..l_b) */
    double r_f;           /* Monte Carlo part (AMC estimate) */
    double psi;           /* Eq. (Delta-st) */
    double eta_star;      /* Eq. (etas-star) */
    double sigma2;        /* empirical variance of the last batch */
    double f_last;        /* Bernstein half-width of the last batch, Eq. (fx) */
} geer_query_stats;

enum {
    GEER_STOP_SAME_NODE = 0,  /* s == t, r = 0 */
    GEER_STOP_NO_WALKS = 1,   /* l_f = l - l_b == 0: nothing left to sample */
    GEER_STOP_BERNSTEIN = 2,  /* f(eta, sigma^2, psi, delta/tau) <= eps/2 */
    GEER_STOP_CAP = 3         /* batch tau reached (eta >= eta*, Hoeffding) */
};

/* Fill *p with the defaults listed above. */
geer_status geer_params_default(geer_params *p);

/* geer_graph_create flags */
enum {
    GEER_GRAPH_TRUSTED = 1u << 0,          /* skip the canonical-form and connectivity checks */
    GEER_GRAPH_WIDE_WALK_RECORDS = 1u << 1 /* 16-byte walk records even where 8 bytes fit */
};

/* Copy a canonical CSR graph to the current HIP device.
 * n: node count (>= 2).  row_ptr: host int32[n+1], row_ptr[0] == 0, non-decreasing.
 * col_idx: host int32[row_ptr[n]].  flags: GEER_GRAPH_* (0 for defaults);
 * GEER_GRAPH_TRUSTED skips the O(nnz log d) canonical-form and connectivity
 * checks (the caller vouches for them).  Besides the CSR the device copy holds
 * one walk record per CSR entry (neighbour, its row start and its degree):
 * 8 bytes when the bit widths of n, nnz and the largest degree add up to at
 * most 64, else 16 bytes.  Returns GEER_E_GRAPH / GEER_E_NOT_CONNECTED for
 * invalid input, GEER_E_INVALID_ARG for unknown flags. */
geer_status geer_graph_create(int32_t n, const int32_t *row_ptr, const int32_t *col_idx,
                              uint32_t flags, geer_graph **out);

/* Free the graph and all device memory it owns.  NULL is ignored. */
void geer_graph_destroy(geer_graph *g);

/* lambda = max(|lambda_2|, |lambda_n|) of P (Theorem 3.1), a per-graph
 * preprocessing value (Section 3.1).  Must satisfy 0 <= lambda < 1
 * (lambda >= 1 -> GEER_E_BIPARTITE). */
geer_status geer_graph_set_lambda(geer_graph *g, double lambda);
geer_status geer_graph_get_lambda(const geer_graph *g, double *lambda_out);

/* Estimate lambda on the GPU by Lanczos on D^-1/2 A D^-1/2 with the top
 * eigenvector sqrt(d) deflated, full reorthogonalisation, and the extreme Ritz
 * values widened by their residual norms (a conservative upper estimate).
 * Stores the value in the graph (as geer_graph_set_lambda) and returns it.
 * max_iter: Krylov dimension (e.g. 300).  tol: stop once both extreme
 * residual norms are below tol. */
geer_status geer_graph_compute_lambda(geer_graph *g, int32_t max_iter, double tol,
                                      uint64_t seed, double *lambda_out);

/* Graph facts: n, nnz (directed CSR entries), max degree. */
geer_status geer_graph_info(const geer_graph *g, int32_t *n, int64_t *nnz, int32_t *max_degree);

/* Answer nq queries (Algorithm 3).  s, t: host int32[nq]; eps: host double[nq]
 * (each > 0, finite).  params may be NULL (defaults).  r_out: host double[nq].
 * stats: host geer_query_stats[nq] or NULL.  Blocks until the results are in
 * host memory. */
geer_status geer_query(geer_graph *g, int64_t nq, const int32_t *s, const int32_t *t,
                       const double *eps, const geer_params *params, double *r_out,
                       geer_query_stats *stats);

/* As geer_query with device inputs and outputs, enqueued on params->stream
 * (or the library stream).  d_s, d_t: device int32[nq]; d_eps: device
 * double[nq]; d_r_out: device double[nq]; d_stats: device
 * geer_query_stats[nq] or NULL.  With params->stream == NULL the work is
 * ordered after everything already queued on the legacy default stream.
 * Node ids and eps are validated on the device;
 * an invalid entry makes the call return GEER_E_INVALID_ARG after the stream
 * has drained (outputs then hold NaN for the invalid queries).  The call
 * returns when the work has finished. */
geer_status geer_query_device(geer_graph *g, int64_t nq, const int32_t *d_s, const int32_t *d_t,
                              const double *d_eps, const geer_params *params, double *d_r_out,
                              geer_query_stats *d_stats);

/* ---- Phase-level entry points (same kernels as geer_query) ------------- */

/* SMM (Algorithm 2) for one batch of nq <= 64 pairs, exactly `hops` products.
 * vec_out: host buffer of n * 2 * nq values (double if GEER_FLAG_FP64_VECTORS
 * is in flags, else float), node-major: entry [v * 2nq + 2j] is s*_j(v) and
 * [v * 2nq + 2j + 1] is t*_j(v).  rb_out: host double[nq], r_b after the hops.
 * top2_out: host double[4 * nq] = (max1 s*, max2 s*, max1 t*, max2 t*) per pair.
 * supp_out: host int64[2 * nq], degree sums over the structural supports of
 * s*_j and t*_j.  Any of the outputs except vec_out may be NULL. */
geer_status geer_smm(geer_graph *g, int32_t nq, const int32_t *s, const int32_t *t, int32_t hops,
                     uint32_t flags, int32_t col_tile, void *vec_out, double *rb_out,
                     double *top2_out, int64_t *supp_out);

/* Record walk node sequences w_1..w_lf with the AMC walk sampler.
 * For walk i: start[i], query id q[i], batch[i], pair index k[i], side[i].
 * trace_out: host int32[nw * lf], row i holds walk i. */
geer_status geer_walk_traces(geer_graph *g, int32_t nw, const int32_t *start, const uint32_t *q,
                             const uint32_t *batch, const uint32_t *k, const uint32_t *side,
                             int32_t lf, uint64_t seed, int32_t *trace_out);

/* Algorithm 1 (AMC) for one pair with caller-supplied non-negative vectors
 * x (for s) and y (for t): host double[n] each (converted to the vector type
 * of flags).  Writes r_f and fills *stats (ell fields set to -1). */
geer_status geer_amc(geer_graph *g, int32_t s, int32_t t, const double *x, const double *y,
                     double eps, int32_t lf, int32_t tau, double delta, uint64_t seed, uint32_t q,
                     uint32_t flags, double *rf_out, geer_query_stats *stats);

/* ---- Allocation-free variant ------------------------------------------- */

/* Bytes of the fixed device scratch array behind geer_amc_device_noalloc
 * (one per device, held until the process ends). */
#define GEER_AMC_SCRATCH_BYTES (16u << 20)

/* For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): geer_amc
 * with device vectors and outputs, which calls no hipMalloc or hipFree and
 * reserves nothing; its scratch (the pair's state, chunk prefix sums and
 * per-chunk partial sums) lives in a static device array of
 * GEER_AMC_SCRATCH_BYTES per device.
 *   d_xy: device array of 2n values (float, or double with
 *         GEER_FLAG_FP64_VECTORS), node-major: d_xy[2v] = x(v), d_xy[2v+1] = y(v);
 *         finite and non-negative (else GEER_E_INVALID_ARG).
 *   d_rf_out: device double[1] <- r_f.  d_stats: device geer_query_stats[1]
 *         or NULL (ell fields -1).
 *   stream: hipStream_t, or NULL for the library stream.  Returns when done.
 * The results are bit-identical to geer_amc on the same values.  Limit: the
 * largest AMC batch may need at most (GEER_AMC_SCRATCH_BYTES - 16384) / 16
 * chunks of 32 walk pairs (about 3.4e7 walk pairs); a larger one returns
 * GEER_E_OOM before any walk is run.  Every call on a device shares that
 * device's array and overwrites what the last call left there: calls that
 * overlap on one device (two host threads, two streams) race and must be
 * serialised by the caller. */
geer_status geer_amc_device_noalloc(geer_graph *g, int32_t s, int32_t t, const void *d_xy,
                                    double eps, int32_t lf, int32_t tau, double delta,
                                    uint64_t seed, uint32_t q, uint32_t flags, void *stream,
                                    double *d_rf_out, geer_query_stats *d_stats);

/* ---- Learned scheduler ------------------------------------------------- */

/* A 3-layer MLP (GEER_MLP_FEATURES -> 64 -> 64 -> 3, ReLU) that predicts, per
 * pair, the SMM depth l_b, the AMC batch count tau and log10 of the absolute
 * error.  Used by GEER_SCHEDULE_LEARNED; pairs whose predicted error exceeds
 * eps or whose per-pair structural features (features 0..8) leave the
 * training range widened by a tenth of its span use the greedy switch of
 * Eq. (smm-amc).  The predicted depth is guarded by exact graph quantities: at
 * least one product when l >= 1, and two when a lower bound of the first walk
 * batch after one product exceeds the hop-2 cost (rho2 times the neighbour
 * degree sums of s and t).  The estimator (l, eta*, the stop rule, delta) is
 * unchanged, so the guarantee of Theorem 3.2 holds for any prediction.
 * Parameters: FP32 master copy, BF16 copy for inference; layout row-major
 * W1[F][64], b1[64], W2[64][64], b2[64], W3[64][3], b3[3].
 * Features (raw, per pair): log2 d(s), log2 d(t), l/16, log2(1 + sum of the
 * neighbour degrees of s), same for t, log2 of the smallest neighbour degree
 * of s, same for t, edge(s,t), log2(1 + common neighbours),
 * log2(1/(1-lambda)), log2 eps, log2 rho2, log2 rhod (cost ratios of the
 * graph, geer_graph_set_costs), log2(max(psi_1, 2^-40) / eps) with psi_1 the
 * Eq. (Delta-st) bound after one product (l_f = l - 1; max1 = 1/(smallest
 * neighbour degree), max2 = 1/(second smallest) or 0 when the degree is 1;
 * psi_1 = 0 when l <= 1). */
#define GEER_MLP_FEATURES 14
#define GEER_MLP_HIDDEN 64
#define GEER_MLP_OUTPUTS 3
#define GEER_MLP_PARAMS (14 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3)

/* New model with He-uniform weights from `seed` (host memory; device copies
 * are made on first use on the current device). */
geer_status geer_model_create(uint64_t seed, geer_model **out);
void geer_model_free(geer_model *m);
/* Checkpoint: weights, Adam moments, step count, seed and feature
 * normalisation; training resumes from a loaded model. */
geer_status geer_model_save(const geer_model *m, const char *path);
geer_status geer_model_load(const char *path, geer_model **out);
/* count must be GEER_MLP_PARAMS.  set_params resets the optimiser state. */
geer_status geer_model_get_params(const geer_model *m, float *out, int64_t count);
geer_status geer_model_set_params(geer_model *m, const float *in, int64_t count);
/* Feature normalisation z = (x - mean) / stdev and the training range [lo, hi]
 * (host float[GEER_MLP_FEATURES] each). */
geer_status geer_model_set_norm(geer_model *m, const float *mean, const float *stdev,
                                const float *lo, const float *hi);
/* Cost ratios used as features: rho2 = cost of one unit of hop-2 push work,
 * rhod = cost of one dense hop of a 64-pair batch divided by 64, both in
 * units of geer_tuning.ns_per_walk_step (geer_autotune measures them).
 * Stored rounded to the nearest power of sqrt(2), so timing noise of a few
 * percent does not change the learned schedule or any answer: ratios within
 * a factor 2^(1/8) of a grid point give bit-identical results.  Both must be
 * positive and finite (else GEER_E_INVALID_ARG). */
geer_status geer_graph_set_costs(geer_graph *g, double rho2, double rhod);
/* Raw features of nq pairs: host float[nq * GEER_MLP_FEATURES]. */
geer_status geer_features(geer_graph *g, int64_t nq, const int32_t *s, const int32_t *t,
                          const double *eps, float *feat_out);
/* Forward pass on normalised inputs x (host float[nb * F]) -> y (host
 * float[nb * 3]), with the FP32 weights or (use_bf16 != 0) the BF16 copy. */
geer_status geer_mlp_forward(geer_model *m, int64_t nb, const float *x, int32_t use_bf16,
                             float *y_out);
/* Gradient of the weighted squared loss mean_b sum_o w[b,o] (yhat - y)^2 of
 * one minibatch (nb <= 64) at the current FP32 weights: host float[PARAMS]. */
geer_status geer_mlp_grad(geer_model *m, int32_t nb, const float *x, const float *y,
                          const float *w, float *grad_out);
/* `steps` Adam steps (lr, beta1 0.9, beta2 0.999) on minibatches of `batch`
 * (<= 64) samples of (x, y, w) (n samples, normalised inputs).  Minibatch
 * indices come from `order` (host int64[steps * batch]) or, if NULL, from a
 * counter-based hash of (model seed, step, slot).  loss_out (nullable):
 * host float[steps], the minibatch loss before each update. */
geer_status geer_mlp_train(geer_model *m, int64_t n, const float *x, const float *y,
                           const float *w, int32_t steps, int32_t batch, double lr,
                           const int64_t *order, float *loss_out);

/* ---- Autotuner ---------------------------------------------------------- */

typedef struct geer_tuning {
    int32_t col_tile;          /* fastest SpMM column tile (32, 64 or 128) */
    int32_t from_cache;        /* 1 if read from the cache file */
    double ns_per_walk_step;   /* the cost unit: one walk step of a pair stopped after one
                                  product whose rows of s and t have at most 256 entries (no
                                  vector read); steps that read SMM vectors cost about twice
                                  as much */
    double ns_per_hop2_unit;   /* one unit of sparse hop-2 work (one CSR entry of one column) */
    double ns_per_dense_hop;   /* one dense hop of a 64-pair batch */
    double rho2, rhod;         /* the cost ratios as stored by geer_graph_set_costs
                                  (rounded to a power of sqrt(2)) */
} geer_tuning;

/* Time the SpMM column tiles and measure the unit costs of the phases on a
 * sample of pairs (host arrays, nq >= 64 recommended; lambda must be set),
 * then store the best tile (used when geer_params.col_tile == 0) and the
 * cost ratios in the graph.  cache_path (nullable): a text file keyed by
 * (n, nnz, max degree, device name); an entry found there is used instead
 * of measuring, and new measurements are appended. */
geer_status geer_autotune(geer_graph *g, int64_t nq, const int32_t *s, const int32_t *t,
                          const double *eps, const char *cache_path, geer_tuning *out);

/* ---- Kernel timing (HIP events on the stream each kernel runs on) ------- */

/* One record per kernel kind: launches, summed event-timed duration, and
 * the algorithmic bytes the launches had to move (SpMM hops: row offsets,
 * column indices, the gathered vector rows once, the written rows once and
 * the inverse degrees of the rows covered; walks: one walk record per step
 * plus the pair's two vector values on steps that read them). */
typedef struct geer_kernel_profile {
    char name[32];
    int64_t launches;
    double total_ms;
    double alg_bytes;
    double work_units;   /* SpMM: CSR entries x active columns; walks: steps */
} geer_kernel_profile;

/* Start (on != 0) or stop timing on this graph; starting clears the records. */
geer_status geer_profile_enable(geer_graph *g, int32_t on);

/* Copy up to cap records (waits for the timed work to finish). */
geer_status geer_profile_read(geer_graph *g, geer_kernel_profile *out, int32_t cap,
                              int32_t *count);

/* Thread-local description of the last non-OK status on this thread. */
const char *geer_last_error(void);

/* Library version string. */
const char *geer_version(void);

#ifdef __cplusplus
}
#endif

#endif /* GEER_H */
