"""Pins for the CPU checker: each test ties part of it to something other
than itself -- printed values of the paper, closed forms, invariants the
paper proves, library routines, an independent Philox implementation and
brute force on tiny graphs.
"""

import os
import shutil
import subprocess

import numpy as np
import pytest

import oracle
from paper_2312_06123_amd import inputs as I

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _dense_adj(g):
    A = np.zeros((g.n, g.n))
    for v in range(g.n):
        A[v, g.col_idx[g.row_ptr[v]:g.row_ptr[v + 1]]] = 1.0
    return A


def _bfs_dist(g, s):
    dist = np.full(g.n, -1)
    dist[s] = 0
    frontier = [s]
    while frontier:
        nxt = []
        for u in frontier:
            for v in g.col_idx[g.row_ptr[u]:g.row_ptr[u + 1]]:
                if dist[v] < 0:
                    dist[v] = dist[u] + 1
                    nxt.append(v)
        frontier = nxt
    return dist


def _small_graphs():
    return [
        I.complete_graph(7),
        I.cycle_graph(9),
        I.lollipop_graph(5, 4),
        I.erdos_renyi_path(40, 4, 7),
        I.chung_lu(300, 2.1, 6, 3),
    ]


# ---------------------------------------------------------------------------
# Philox4x32-10
# ---------------------------------------------------------------------------

def test_philox_known_answers():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "philox4x32_10_kat.txt"))
            if l.strip() and not l.startswith("#")]
    assert len(rows) == 3
    for r in rows:
        vals = [int(x, 16) for x in r]
        out = oracle.philox4x32_10(vals[0:4], vals[4:6])
        assert out.tolist() == vals[6:10]


def test_philox_matches_rocrand_engine(tmp_path):
    hipcc = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
    if not os.path.exists(hipcc):
        pytest.skip("hipcc not available")
    exe = tmp_path / "probe"
    src = os.path.join(os.path.dirname(__file__), "philox_rocrand_probe.cpp")
    subprocess.check_call([hipcc, "-O1", "-o", str(exe), src], stdout=subprocess.DEVNULL,
                          stderr=subprocess.DEVNULL)
    rng = np.random.default_rng(5)
    ctrs = rng.integers(0, 2**32, size=(200, 6), dtype=np.uint64)
    ctrs[:, 1] %= 2**30  # the engine's 64-bit offset arithmetic needs 4*(c1:c0) < 2^64
    text = "\n".join(" ".join("%x" % v for v in row) for row in ctrs) + "\n"
    out = subprocess.run([str(exe)], input=text, capture_output=True, text=True, check=True).stdout
    got = [[int(x, 16) for x in l.split()] for l in out.strip().splitlines()]
    for row, ref in zip(ctrs, got):
        mine = oracle.philox4x32_10([int(v) for v in row[:4]], [int(v) for v in row[4:6]])
        assert mine.tolist() == ref


# ---------------------------------------------------------------------------
# Walk sampler
# ---------------------------------------------------------------------------

def test_walk_traces_are_walks_and_deterministic():
    g = I.chung_lu(500, 2.1, 8, 11)
    for k in range(20):
        tr = oracle.walk_trace(g.row_ptr, g.col_idx, 3, 25, 99, 7, 1, k, k & 1)
        prev = 3
        for u in tr:
            assert u in g.col_idx[g.row_ptr[prev]:g.row_ptr[prev + 1]]
            prev = u
        tr2 = oracle.walk_trace(g.row_ptr, g.col_idx, 3, 25, 99, 7, 1, k, k & 1)
        assert np.array_equal(tr, tr2)


def test_walk_first_step_uniform_over_neighbours():
    # chi-square test that the first step is uniform over the 7 neighbours of
    # the star centre (draw mod d is unbiased up to d / 2^32)
    g = I.star_graph(7)
    counts = np.zeros(g.n)
    for k in range(7000):
        counts[oracle.walk_trace(g.row_ptr, g.col_idx, 0, 1, 123, 0, 0, k, 0)[0]] += 1
    obs = counts[1:]
    chi2 = ((obs - 1000.0) ** 2 / 1000.0).sum()
    assert counts[0] == 0
    assert chi2 < 22.46  # 6 dof, p = 0.001


def test_walk_counter_fields_are_independent_streams():
    g = I.complete_graph(50)
    base = oracle.walk_trace(g.row_ptr, g.col_idx, 0, 16, 1, 2, 3, 4, 0)
    for args in [(1, 2, 3, 4, 1), (1, 2, 3, 5, 0), (1, 2, 4, 4, 0), (1, 3, 3, 4, 0), (2, 2, 3, 4, 0)]:
        other = oracle.walk_trace(g.row_ptr, g.col_idx, 0, 16, *args)
        assert not np.array_equal(base, other)


# ---------------------------------------------------------------------------
# SMM products and the truncated series
# ---------------------------------------------------------------------------

def test_toy_path_counts_match_printed_table():
    lines = {l.split()[0]: l.split()[1:] for l in open(os.path.join(GOLDEN, "toy_running_example.txt"))
             if l.strip() and not l.startswith("#")}
    edges = np.array([[int(a) for a in e.split("-")] for e in lines["edges"]])
    g = I.from_edges(11, edges)
    deg = g.degrees().astype(float)
    for who, key in (("s", "paths_s"), ("t", "paths_t")):
        x = np.zeros(g.n)
        x[int(lines[who][0])] = 1.0
        got = []
        for _ in lines["lf"]:
            # A x = D (P x): the checker's product with P, rescaled to walk counts
            x = deg * oracle.smm_hop(g.row_ptr, g.col_idx, x)
            got.append(int(round(x.sum())))
        assert got == [int(v) for v in lines[key]]


@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: g.name)
def test_smm_hop_is_transition_product(g):
    A = _dense_adj(g)
    P = A / A.sum(axis=1, keepdims=True)
    x = np.random.default_rng(1).random(g.n)
    assert np.allclose(oracle.smm_hop(g.row_ptr, g.col_idx, x), P @ x, rtol=1e-13, atol=0)


@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: g.name)
def test_smm_invariants_and_supports(g):
    deg = g.degrees().astype(float)
    A = _dense_adj(g)
    s, t = 0, g.n - 1
    for hops in range(0, 7):
        x, y, sx, sy, rb = oracle.smm_vectors(g.row_ptr, g.col_idx, s, t, hops)
        # mass: sum_v d(v) x(v) = d(s)
        assert abs((deg * x).sum() - deg[s]) < 1e-12 * deg[s]
        assert abs((deg * y).sum() - deg[t]) < 1e-12 * deg[t]
        # reversibility: d(t) p_i(t,s) = d(s) p_i(s,t)
        assert abs(deg[t] * x[t] - deg[s] * y[s]) < 1e-13
        # structural support = nonzero pattern of A^hops e_s (integer powers)
        ps = np.linalg.matrix_power(A, hops)[:, s] > 0
        pt = np.linalg.matrix_power(A, hops)[:, t] > 0
        assert np.array_equal(sx, ps) and np.array_equal(sy, pt)


def test_series_complete_graph_closed_form():
    # P = (J - I)/(n-1): every non-trivial eigenvalue is -1/(n-1), so
    # r_l = (2/n) (1 - (-1/(n-1))^(l+1))
    for n in (4, 6, 11):
        g = I.complete_graph(n)
        for l in range(0, 9):
            r = oracle.series(g.row_ptr, g.col_idx, [0], [n - 1], [l])[0]
            assert abs(r - (2.0 / n) * (1 - (-1.0 / (n - 1)) ** (l + 1))) < 1e-14


def test_series_odd_cycle_spectral_closed_form():
    # C_n: p_i(u,v) = (1/n) sum_k cos(2 pi k (u - v)/n) cos(2 pi k/n)^i
    n = 11
    g = I.cycle_graph(n)
    k = np.arange(n)
    lam = np.cos(2 * np.pi * k / n)
    for dist in (1, 3, 5):
        s, t = 0, dist
        for l in (0, 1, 2, 5, 12):
            terms = []
            for i in range(l + 1):
                pss = np.mean(lam ** i)
                pst = np.mean(np.cos(2 * np.pi * k * dist / n) * lam ** i)
                terms.append((2 * pss - 2 * pst) / 2.0)
            r = oracle.series(g.row_ptr, g.col_idx, [s], [t], [l])[0]
            assert abs(r - sum(terms)) < 1e-13


@pytest.mark.parametrize("g", _small_graphs()[:4], ids=lambda g: g.name)
def test_series_even_terms_nonnegative_and_tail_bound(g):
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    deg = g.degrees()
    rng = np.random.default_rng(3)
    for _ in range(6):
        s, t = rng.choice(g.n, 2, replace=False)
        r = oracle.exact_pinv(g.row_ptr, g.col_idx, s, t)
        prev = oracle.series(g.row_ptr, g.col_idx, [s], [t], [0])[0]
        for l in range(1, 25):
            cur = oracle.series(g.row_ptr, g.col_idx, [s], [t], [l])[0]
            if l % 2 == 0:
                assert cur - prev >= -1e-15  # Eq. (pflambda): even-power terms are >= 0
            tail = lam ** (l + 1) / (1 - lam) * (1.0 / deg[s] + 1.0 / deg[t])
            assert abs(r - cur) <= tail + 1e-12  # proof of Theorem 3.1
            prev = cur


# ---------------------------------------------------------------------------
# Exact resistance
# ---------------------------------------------------------------------------

def test_exact_closed_forms():
    cases = [
        (I.complete_graph(7), 0, 5, 2.0 / 7),
        (I.cycle_graph(9), 0, 3, 3 * 6 / 9),
        (I.cycle_graph(12), 2, 7, 5 * 7 / 12),
        (I.path_graph(8), 1, 6, 5.0),
        (I.star_graph(6), 1, 2, 2.0),
        (I.complete_bipartite(3, 5), 0, 1, 2.0 / 5),      # same side of the 3-part
        (I.complete_bipartite(3, 5), 3, 4, 2.0 / 3),      # same side of the 5-part
        (I.complete_bipartite(3, 5), 0, 3, 7.0 / 15),     # across: (a+b-1)/(ab)
        (I.lollipop_graph(6, 3), 5, 8, 3.0),              # tail is a path of bridges
    ]
    for g, s, t, want in cases:
        assert abs(oracle.exact_pinv(g.row_ptr, g.col_idx, s, t) - want) < 1e-10, g.name
        r, _ = oracle.exact_cg(g.row_ptr, g.col_idx, [s], [t])
        assert abs(r[0] - want) < 1e-10, g.name


@pytest.mark.parametrize("g", _small_graphs(), ids=lambda g: g.name)
def test_exact_foster_triangle_and_distance(g):
    e = g.edges()
    Lp = np.linalg.pinv(oracle.laplacian_dense(g.row_ptr, g.col_idx), hermitian=True)
    dg = np.diag(Lp)
    R = dg[:, None] + dg[None, :] - 2 * Lp
    # Foster's theorem: sum over edges of r = n - 1
    assert abs(R[e[:, 0], e[:, 1]].sum() - (g.n - 1)) < 1e-8
    # metric: triangle inequality; r <= shortest-path distance
    idx = np.random.default_rng(0).choice(g.n, size=(200, 3))
    a, b, c = idx.T
    assert np.all(R[a, c] <= R[a, b] + R[b, c] + 1e-9)
    for s in range(0, g.n, max(1, g.n // 7)):
        dist = _bfs_dist(g, s)
        assert np.all(R[s] <= dist + 1e-9)
    # CG and pseudo-inverse agree
    rng = np.random.default_rng(1)
    s = rng.integers(0, g.n, 30).astype(np.int32)
    t = ((s + rng.integers(1, g.n, 30)) % g.n).astype(np.int32)
    r, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s, t)
    assert np.allclose(r, R[s, t], rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# lambda and l
# ---------------------------------------------------------------------------

def test_lambda_closed_forms():
    for n in (5, 8):
        g = I.complete_graph(n)
        assert abs(oracle.lambda_dense(g.row_ptr, g.col_idx) - 1.0 / (n - 1)) < 1e-12
    for n in (7, 9, 15):
        g = I.cycle_graph(n)
        assert abs(oracle.lambda_dense(g.row_ptr, g.col_idx) - np.cos(np.pi / n)) < 1e-12
    g = I.cycle_graph(8)  # bipartite: lambda_n = -1
    assert abs(oracle.lambda_dense(g.row_ptr, g.col_idx) - 1.0) < 1e-12


@pytest.mark.parametrize("g", _small_graphs()[2:], ids=lambda g: g.name)
def test_lambda_arpack_matches_dense(g):
    assert abs(oracle.lambda_arpack(g.row_ptr, g.col_idx)
               - oracle.lambda_dense(g.row_ptr, g.col_idx)) < 1e-8


@pytest.mark.parametrize("g", _small_graphs()[:4], ids=lambda g: g.name)
def test_ell_meets_theorem_bound(g):
    # Theorem 3.1: with l from Eq. (ell), |r - r_l| <= eps/2
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    deg = g.degrees()
    rng = np.random.default_rng(2)
    for eps in (0.5, 0.1, 0.02, 1e-3):
        for _ in range(8):
            s, t = rng.choice(g.n, 2, replace=False)
            l = oracle.ell(deg[s], deg[t], eps, lam)
            assert l >= 0
            r = oracle.exact_pinv(g.row_ptr, g.col_idx, s, t)
            rl = oracle.series(g.row_ptr, g.col_idx, [s], [t], [l])[0]
            assert abs(r - rl) <= eps / 2 + 1e-12
            # Eq. (ell) never exceeds the degree-free length of Eq. (old-ell)
            assert l <= oracle.ell_peng(eps, lam)


@pytest.mark.parametrize("g", _small_graphs()[:4], ids=lambda g: g.name)
def test_peng_ell_bound_and_geer_variant(g):
    # Eq. (old-ell): one length for every pair, also within eps/2 of r; at
    # d(s) = d(t) = 1 it coincides with Eq. (ell)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    rng = np.random.default_rng(3)
    for eps in (0.5, 0.1, 0.02):
        lp = oracle.ell_peng(eps, lam)
        assert lp == oracle.ell(1, 1, eps, lam)
        for _ in range(6):
            s, t = rng.choice(g.n, 2, replace=False)
            r = oracle.exact_pinv(g.row_ptr, g.col_idx, s, t)
            rl = oracle.series(g.row_ptr, g.col_idx, [s], [t], [lp])[0]
            assert abs(r - rl) <= eps / 2 + 1e-12
    # GEER with the variant length: every pair gets l = Eq. (old-ell), and the
    # SMM-only run (l_b = l) is the truncated series at that length
    s, t = (np.array(x, dtype=np.int32) for x in zip(*[rng.choice(g.n, 2, replace=False) for _ in range(10)]))
    r, st = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.1, lam, seed=4, ell_rule="peng",
                        schedule="fixed", fixed_lb=10 ** 6)
    assert np.all(st["ell"] == oracle.ell_peng(0.1, lam))
    rl = oracle.series(g.row_ptr, g.col_idx, s, t, st["ell"])
    assert np.allclose(r, rl, rtol=1e-12, atol=1e-14)


def test_ell_monotone_and_clamped():
    assert oracle.ell(1, 1, 10.0, 0.5) == 0
    assert oracle.ell(3, 4, 0.1, 0.0) == 0
    prev = 0
    for eps in (1.0, 0.5, 0.2, 0.1, 0.05, 0.02, 0.01):
        cur = oracle.ell(5, 7, eps, 0.8)
        assert cur >= prev
        prev = cur
    assert oracle.ell(5, 7, 0.05, 0.9) >= oracle.ell(5, 7, 0.05, 0.8)
    assert oracle.ell(50, 70, 0.05, 0.8) <= oracle.ell(5, 7, 0.05, 0.8)


# ---------------------------------------------------------------------------
# AMC: bounds, unbiasedness, budgets
# ---------------------------------------------------------------------------

def test_walk_sum_bound_and_unbiasedness():
    # Lemma 3.3: |Z_k| <= psi/2 for every sample; Eq. (x-exp): E[Z_k] = q(s,t),
    # where q = r_l - r_b(l_b) by Eq. (2-parts)
    g = I.chung_lu(400, 2.1, 8, 21)
    deg = g.degrees()
    s, t = 5, 301
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    for lb in (0, 1, 2, 4):
        lf = 6
        x, y, _, _, rb = oracle.smm_vectors(g.row_ptr, g.col_idx, s, t, lb)
        m1s, m2s = oracle.top2(x)
        m1t, m2t = oracle.top2(y)
        psi = oracle.psi(lf, m1s, m2s, m1t, m2t, deg[s], deg[t])
        z = oracle.amc_samples(g.row_ptr, g.col_idx, s, t, x, y, lf, 77, 0, 0, 40000)
        assert np.all(np.abs(z) <= psi / 2 * (1 + 1e-12))
        q = oracle.series(g.row_ptr, g.col_idx, [s], [t], [lb + lf])[0] - rb
        se = z.std() / np.sqrt(z.size)
        assert abs(z.mean() - q) < 4.5 * se + 1e-12, (lb, z.mean(), q, se)
    assert lam < 1


def test_hoeffding_cap_and_walk_budget():
    # proof of Theorem 3.2: 2 exp(-eta* eps^2 / (2 psi^2)) = delta / tau
    for psi in (0.01, 0.3, 4.0):
        for eps in (0.5, 0.05):
            for tau in (1, 3, 5, 8):
                es = oracle.eta_star(psi, eps, tau, 0.01)
                assert abs(2 * np.exp(-es * eps ** 2 / (2 * psi ** 2)) - 0.01 / tau) < 1e-12
                e1 = oracle.eta1(es, tau)
                # the last batch reaches the cap: 2^(tau-1) eta_1 >= eta*
                assert e1 * 2 ** (tau - 1) >= es - 1e-9
                h = oracle.h_budget(es, tau)
                # Section 3.3.2: h = (2^tau - 1) eta_1 < 2 eta* (up to the ceiling)
                assert h == (2 ** tau - 1) * e1
                assert h <= 2 * es + 2 ** tau


def test_bernstein_shape():
    # Eq. (fx): decreasing in the sample count, increasing in variance and range
    f = [oracle.bernstein(nz, 0.1, 1.0, 0.01) for nz in (10, 100, 1000)]
    assert f[0] > f[1] > f[2]
    assert oracle.bernstein(100, 0.2, 1.0, 0.01) > oracle.bernstein(100, 0.1, 1.0, 0.01)
    assert oracle.bernstein(100, 0.1, 2.0, 0.01) > oracle.bernstein(100, 0.1, 1.0, 0.01)
    # zero variance leaves only the range term
    assert abs(oracle.bernstein(50, 0.0, 1.0, 0.03) - 3 * np.log(100) / 50) < 1e-15


def test_top2_counts_repeats():
    assert oracle.top2(np.array([0.0, 3.0, 1.0, 3.0])) == (3.0, 3.0)
    assert oracle.top2(np.array([0.0, 1.0, 0.0])) == (1.0, 0.0)


# ---------------------------------------------------------------------------
# GEER end to end
# ---------------------------------------------------------------------------

def test_geer_smm_only_is_within_half_eps():
    # l_b = l: no walks; Theorem 3.1 alone gives |r_b - r| <= eps/2
    g = I.erdos_renyi_path(200, 6, 4)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 60, 9)
    r, st = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.05, lam, schedule="fixed",
                        fixed_lb=1000)
    ex = oracle.exact_pinv(g.row_ptr, g.col_idx, s, t)
    assert np.all(st["walk_pairs"] == 0)
    assert np.all(np.abs(r - ex) <= 0.025 + 1e-12)


@pytest.mark.parametrize("schedule,lb", [("greedy", None), ("fixed", 0), ("fixed", 2)])
def test_geer_coverage(schedule, lb):
    # Theorem 3.2 / Section 4.2: |r' - r| <= eps with probability >= 1 - delta
    g = I.chung_lu(600, 2.1, 10, 31)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 400, 41)
    eps = 0.2
    r, st = oracle.geer(g.row_ptr, g.col_idx, s, t, eps, lam, seed=5, schedule=schedule,
                        fixed_lb=lb)
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s, t)
    cover = np.mean(np.abs(r - ex) <= eps)
    assert cover >= 0.99
    if schedule == "fixed":
        assert np.all(st["ell_b"] == np.minimum(lb, st["ell"]))
    else:
        # the greedy rule stopped at l or once SMM's next-hop cost exceeded h
        deg = g.degrees()
        for i in range(len(s)):
            rec = st[i]
            if rec["ell_b"] < rec["ell"] and rec["ell_b"] > 0:
                assert rec["supp_sum"] > oracle.h_budget(rec["eta_star"], 5) - 1e-9


def test_geer_same_node_and_stats():
    g = I.complete_graph(6)
    r, st = oracle.geer(g.row_ptr, g.col_idx, [2, 1], [2, 4], 0.1, 0.2)
    assert r[0] == 0.0 and st[0]["ell"] == 0
    assert abs(r[1] - 2 / 6) <= 0.1


# ---------------------------------------------------------------------------
# learned-scheduler network reference
# ---------------------------------------------------------------------------

def test_mlp_reference_gradient_matches_finite_differences():
    from oracle import mlp

    rng = np.random.default_rng(0)
    p = rng.normal(0, 0.3, mlp.P)
    X = rng.normal(0, 1, (9, mlp.F))
    Y = rng.normal(0, 1, (9, mlp.O))
    Wt = rng.random((9, mlp.O))
    g = mlp.grad(p, X, Y, Wt)
    h = 1e-6
    for k in rng.choice(mlp.P, 60, replace=False):
        e = np.zeros(mlp.P)
        e[k] = h
        fd = (mlp.loss(p + e, X, Y, Wt) - mlp.loss(p - e, X, Y, Wt)) / (2 * h)
        assert abs(fd - g[k]) <= 1e-6 * max(1.0, abs(fd))


def test_mlp_reference_adam_reduces_loss():
    from oracle import mlp

    rng = np.random.default_rng(1)
    X = rng.normal(0, 1, (64, mlp.F))
    Y = np.stack([X[:, 0] + 2 * X[:, 1], X[:, 2] ** 2, np.sin(X[:, 3])], axis=1)
    Wt = np.ones_like(Y)
    p = rng.normal(0, 0.2, mlp.P)
    m = np.zeros(mlp.P)
    v = np.zeros(mlp.P)
    l0 = mlp.loss(p, X, Y, Wt)
    for step in range(1, 301):
        p, m, v = mlp.adam_step(p, m, v, mlp.grad(p, X, Y, Wt), step, 3e-3)
    assert mlp.loss(p, X, Y, Wt) < 0.2 * l0


def test_geer_per_pair_tau_matches_uniform_tau():
    g = I.erdos_renyi_path(300, 6, 44)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 40, 45)
    for tau in (1, 3, 5):
        r1, st1 = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.2, lam, tau=tau, seed=2)
        r2, st2 = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.2, lam, tau=5, seed=2,
                              tau_per_pair=np.full(len(s), tau))
        assert np.array_equal(r1, r2) and np.array_equal(st1["batches_run"], st2["batches_run"])


# ---------------------------------------------------------------------------
# Two-sided pins: each of these fails when the checker's formula is off in
# either direction (a length one too long, a bound too loose or too tight, a
# stop one hop late), not only when it is unsafe.
# ---------------------------------------------------------------------------

def _tail(lam, l, ds, dt):
    # the bound at the end of the proof of Theorem 3.1:
    # |r - r_l| <= lam^(l+1) / (1 - lam) * (1/d(s) + 1/d(t))
    return lam ** (l + 1) / (1.0 - lam) * (1.0 / ds + 1.0 / dt)


def test_ell_is_smallest_length_meeting_the_tail_bound():
    # Eq. (ell) solves the proof's tail bound for l: the returned l meets
    # tail <= eps/2 and l - 1 does not (whenever l >= 1)
    checked = 0
    for ds in (1, 2, 3, 7, 50, 1000):
        for dt in (1, 4, 13, 300):
            for eps in (0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 1e-3):
                for lam in (0.1, 0.3, 0.5, 0.7, 0.866, 0.9, 0.97, 0.999):
                    l = oracle.ell(ds, dt, eps, lam)
                    assert l >= 0
                    assert _tail(lam, l, ds, dt) <= eps / 2 * (1 + 1e-12)
                    if l >= 1:
                        prev = _tail(lam, l - 1, ds, dt)
                        if abs(prev / (eps / 2) - 1.0) < 1e-9:
                            continue  # exact tie: either length is a correct reading
                        assert prev > eps / 2, (ds, dt, eps, lam, l)
                        checked += 1
    assert checked > 600


def test_peng_ell_is_smallest_length_meeting_its_bound():
    # Eq. (old-ell) is the same bound with 1/d(s) + 1/d(t) replaced by 2
    checked = 0
    for eps in (0.5, 0.2, 0.1, 0.05, 0.02, 0.01, 1e-3):
        for lam in (0.1, 0.3, 0.5, 0.7, 0.866, 0.9, 0.97, 0.999):
            l = oracle.ell_peng(eps, lam)
            assert _tail(lam, l, 1, 1) <= eps / 2 * (1 + 1e-12)
            if l >= 1:
                assert _tail(lam, l - 1, 1, 1) > eps / 2
                checked += 1
    assert checked > 40


def _two_paths():
    # b - a - s - t - c - d  with s = 0, a = 1, b = 2, t = 3, c = 4, d = 5:
    # a walk from s can alternate a, b, a, b, ... and one from t c, d, c, ...
    return I.from_edges(6, np.array([[0, 1], [1, 2], [0, 3], [3, 4], [4, 5]]))


@pytest.mark.parametrize("lf,half_psi", [(5, 3 * 0.6 + 2 * 0.25), (7, 4 * 0.6 + 3 * 0.25),
                                         (6, 3 * 0.6 + 3 * 0.25)])
def test_psi_is_attained_by_an_alternating_walk(lf, half_psi):
    # Lemma 3.3's bound is tight: a walk that alternates between the largest
    # and second-largest entries of x collects ceil(lf/2) max1 + floor(lf/2)
    # max2.  Here x = 0.5 at a, 0.3 at b; y = 0.7 at c, 0.2 at d; d(s) = d(t)
    # = 2, so psi/2 = ceil(lf/2) (0.25 + 0.35) + floor(lf/2) (0.15 + 0.1)
    # (the expected values above, worked out by hand).  The largest sampled
    # Z_k must equal psi/2: at odd lf this fixes which of max1 and max2 takes
    # the ceiling, and equality fixes psi from above as well.
    g = _two_paths()
    deg = g.degrees()
    x = np.zeros(6)
    y = np.zeros(6)
    x[1], x[2] = 0.5, 0.3
    y[4], y[5] = 0.7, 0.2
    m1s, m2s = oracle.top2(x)
    m1t, m2t = oracle.top2(y)
    psi = oracle.psi(lf, m1s, m2s, m1t, m2t, deg[0], deg[3])
    assert psi == pytest.approx(2 * half_psi, rel=1e-14)
    z = oracle.amc_samples(g.row_ptr, g.col_idx, 0, 3, x, y, lf, 2024, 0, 0, 20000)
    assert np.all(np.abs(z) <= psi / 2 * (1 + 1e-14))
    assert z.max() == pytest.approx(psi / 2, rel=1e-14)


def test_bernstein_width_brackets_the_normal_quantile():
    # Eq. (fx) at a large sample count: the range term vanishes and the width
    # sqrt(2 var ln(3/delta) / n) must lie between the two-sided normal
    # quantile z_{1-delta/2} sigma / sqrt(n) (the limit any valid bound must
    # reach, central limit theorem) and 1.5 times it (sqrt(2 ln 300) / z_0.995
    # = 1.31).  A two-point distribution {0, psi} with P(psi) = p has
    # variance p (1 - p) psi^2.
    from scipy.stats import norm

    for delta in (0.01, 0.002):
        for p in (0.5, 0.1, 0.01):
            for psi in (1.0, 0.03):
                n = 1e9
                var = p * (1 - p) * psi ** 2
                clt = norm.ppf(1 - delta / 2) * np.sqrt(var / n)
                f = oracle.bernstein(n, var, psi, delta)
                assert clt <= f <= 1.5 * clt, (delta, p, psi, f / clt)


def test_bernstein_width_covers_the_mean_on_small_samples():
    # Lemma 3.2 itself: |Z - E Z| < f(n, var_hat, psi, delta) on at least
    # 1 - delta of repeated experiments, here with skewed two-point samples
    # where the range term matters
    rng = np.random.default_rng(8)
    delta, reps = 0.05, 4000
    for n, p in ((20, 0.05), (50, 0.2), (200, 0.5)):
        zs = (rng.random((reps, n)) < p).astype(np.float64)
        mean = zs.mean(axis=1)
        var = np.maximum(0.0, (zs ** 2).mean(axis=1) - mean ** 2)
        f = np.array([oracle.bernstein(n, v, 1.0, delta) for v in var])
        assert np.mean(np.abs(mean - p) >= f) <= delta


def test_greedy_switch_stops_at_the_first_hop_where_the_rule_holds():
    # Eq. (smm-amc) is checked after every product (repeat-until): the greedy
    # schedule must stop at the first hop l_b at which the support degree sum
    # exceeds h(l - l_b), so the rule held at l_b (or l_b = l) and was false
    # at every hop 1..l_b - 1.  Supports and psi are recomputed hop by hop
    # from the checker's SMM vectors.
    g = I.chung_lu(700, 2.1, 8, 61)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    deg = g.degrees()
    s, t = I.uniform_pairs(g.n, 120, 62)
    tau, delta = 5, 0.01
    deep = 0
    for eps in (0.2, 0.02):
        _, st = oracle.geer(g.row_ptr, g.col_idx, s, t, eps, lam, tau=tau, delta=delta, seed=3)
        for j in range(len(s)):
            l, lb = int(st["ell"][j]), int(st["ell_b"][j])
            if l == 0:
                assert lb == 0
                continue
            assert 1 <= lb <= l
            for hop in range(1, lb + 1):
                x, y, sx, sy, _ = oracle.smm_vectors(g.row_ptr, g.col_idx, s[j], t[j], hop)
                supp = deg[sx].sum() + deg[sy].sum()
                psi = oracle.psi(l - hop, *oracle.top2(x), *oracle.top2(y), deg[s[j]], deg[t[j]])
                h = oracle.h_budget(oracle.eta_star(psi, eps, tau, delta), tau)
                holds = supp > h
                if hop < lb:
                    assert not holds, (eps, j, hop, lb, supp, h)
                elif lb < l:
                    assert holds, (eps, j, hop, supp, h)
            deep += lb >= 2
    assert deep >= 20  # the one-hop-earlier check is exercised


def test_mlp_reference_adam_steps_by_lr_with_bias_correction():
    # Adam (Kingma & Ba, with bias correction): under a constant gradient the
    # corrected moments are m_hat = g and v_hat = g^2 at every step, so each
    # coordinate with a nonzero gradient moves by exactly lr (up to eps / |g|)
    from oracle import mlp

    rng = np.random.default_rng(4)
    p = rng.normal(0, 1, mlp.P)
    # gradients of either sign spanning five decades, all far above eps = 1e-8
    g = rng.choice([-1.0, 1.0], mlp.P) * rng.uniform(1.0, 10.0, mlp.P) * 10.0 ** rng.integers(-3, 2, mlp.P)
    g[::17] = 0.0
    m = np.zeros(mlp.P)
    v = np.zeros(mlp.P)
    lr = 1e-3
    for step in range(1, 6):
        p2, m, v = mlp.adam_step(p, m, v, g, step, lr)
        moved = p - p2
        nz = g != 0
        assert np.allclose(moved[nz], lr * np.sign(g[nz]), rtol=1e-4, atol=0)
        assert np.all(moved[~nz] == 0)
        p = p2
