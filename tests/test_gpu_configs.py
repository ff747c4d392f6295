"""Parity at the shapes of the other workloads (each a module of its own).

  * ER n = 10^4, mean degree 10, 1,000 uniform pairs, eps = 0.1, FP64 vectors
    and sums: every pair replayed by the FP64 checker with the same walks;
    decisions agree on >= 99% of pairs and the answers there to 1e-9;
  * R-MAT scale 22 (a = 0.57, b = c = 0.19), 100,000 pairs (half uniform,
    half degree-proportional), per-pair eps drawn from {0.02, 0.05, 0.1},
    autotuned tile: the greedy schedule, and the learned one both launched
    directly and captured in one hipGraph (bit-identical); stratified samples
    checked against the exact resistance (|r' - r| <= eps, 264 pairs) and
    replayed by the checker; the graph's bit widths exceed 64, so the walks
    run on 16-byte records;
  * the learned checkpoint on a fresh Chung-Lu graph (n = 2 * 10^6, the 1M
    configuration's parameters), 50,000 uniform pairs, eps = 0.05: the model
    applies to most pairs, sampled answers are within eps of the exact
    resistance and equal the checker's run at the same (l_b, tau);
  * R-MAT scale 24 (16 * 2^24 samples, ~5 * 10^8 CSR entries, fully resident),
    10^6 degree-proportional pairs, eps = 0.02, learned schedule, run in
    chunks of 10^5 pairs (walk ids continue across chunks): 24 sampled pairs
    replayed by the checker, 72 checked against the exact resistance.
    Generating the graph takes ~40 s and ~35 GB of host memory.
"""

import os

import numpy as np
import pytest

import oracle
import parity
from paper_2312_06123_amd import inputs as I

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2312_06123_amd.geer")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


# ---------------------------------------------------------------------------
# ER n = 10^4, FP64 throughout
# ---------------------------------------------------------------------------

def test_er10k_fp64_every_pair_replayed():
    g = I.erdos_renyi_path(10_000, 10, 1001)
    assert g.nnz == 100_000
    s, t = I.uniform_pairs(g.n, 1000, 2001)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx) as gg:
        lam = G.geer_graph_compute_lambda(gg.handle, 300, 1e-10, 7)
        p = G.geer_params_default(seed=3001, flags=G.GEER_FLAG_FP64_VECTORS)
        r, st = G.geer_query(gg.handle, s, t, 0.1, p, stats=True)
    ref = oracle.lambda_arpack(g.row_ptr, g.col_idx, tol=1e-12)
    assert ref - 1e-9 <= lam <= ref + 1e-6
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.1, lam, seed=3001)
    cnt = parity.compare(g, s, t, 0.1, lam, st, sto, tau=5, seed=3001, fp64=True, label="er10k fp64")
    assert cnt["agree"] >= 0.99 * len(s)
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s, t, tol=1e-12)
    assert np.mean(np.abs(r - ex) <= 0.1) >= 0.99


# ---------------------------------------------------------------------------
# R-MAT scale 22, mixed eps, uniform + degree-proportional pairs
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rmat22_run():
    g = I.rmat(22, 16, 0.57, 0.19, 0.19, 1003)
    nq = 100_000
    su, tu = I.uniform_pairs(g.n, nq // 2, 2003)
    sd, td = I.degree_pairs(g, nq // 2, 2103)
    s = np.concatenate([su, sd])
    t = np.concatenate([tu, td])
    eps = np.random.default_rng(2203).choice(np.array([0.02, 0.05, 0.1]), nq)
    model = G.Model(path=os.path.join(ROOT, "paper_2312_06123_amd", "data", "scheduler.geermlp"))
    learned = {}
    with G.Graph(g.n, g.row_ptr32(), g.col_idx) as gg:
        lam = G.geer_graph_compute_lambda(gg.handle, 400, 1e-8, 7)
        ts, tt = I.uniform_pairs(g.n, 1024, 2303)
        G.geer_autotune(gg.handle, ts, tt, 0.05)
        r, st = G.geer_query(gg.handle, s, t, eps, G.geer_params_default(seed=3003), stats=True)
        for name, flags in (("direct", 0), ("graph", G.GEER_FLAG_GRAPH_LAUNCH)):
            p = G.geer_params_default(seed=3303, schedule=G.GEER_SCHEDULE_LEARNED,
                                      model=model.handle.value, flags=flags)
            learned[name] = G.geer_query(gg.handle, s, t, eps, p, stats=True)
    model.close()
    # stratified samples per (eps, pair kind): 4 pairs each replayed by the
    # checker, 40 further pairs each checked against the exact resistance
    rng = np.random.default_rng(0)
    sample, cover = [], []
    for e in (0.02, 0.05, 0.1):
        for half in (0, 1):
            idx = np.flatnonzero((eps == e) & ((np.arange(nq) >= nq // 2) == bool(half)))
            pick = rng.choice(idx, 44, replace=False)
            sample.extend(pick[:4].tolist())
            cover.extend(pick[4:].tolist())
    idx = np.concatenate([sample, cover])
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s[idx], t[idx], tol=1e-10)
    exact = dict(zip(idx.tolist(), ex.tolist()))
    return g, s, t, eps, lam, r, st, np.array(sample), np.array(cover), learned, exact


def test_rmat22_coverage_on_stratified_sample(rmat22_run):
    # Definition 2.2: |r' - r| <= eps with probability >= 1 - delta = 0.99;
    # 264 pairs (44 per eps and pair kind) against the exact resistance
    g, s, t, eps, lam, r, st, sample, cover, learned, exact = rmat22_run
    deg = g.degrees()
    assert deg.max() > 100_000  # hub rows span hundreds of segments
    assert np.all(np.isfinite(r))
    idx = np.concatenate([sample, cover])
    ex = np.array([exact[i] for i in idx.tolist()])
    fails = np.abs(r[idx] - ex) > eps[idx]
    print(f"[coverage] rmat22: {len(idx) - fails.sum()}/{len(idx)} within eps; "
          f"max |r' - r| / eps = {np.max(np.abs(r[idx] - ex) / eps[idx]):.3f}", flush=True)
    assert not fails[:len(sample)].any()
    assert fails.sum() <= 0.01 * len(idx)


def test_rmat22_replay_on_sample(rmat22_run):
    g, s, t, eps, lam, r, st, sample, cover, learned, exact = rmat22_run
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s[sample], t[sample], eps[sample], lam, seed=3003,
                          qid=sample)
    parity.compare(g, s[sample], t[sample], eps[sample], lam, st[sample], sto, tau=5, seed=3003,
                   qid=sample, label="rmat22 greedy")


def test_rmat22_learned_graph_launch(rmat22_run):
    # the learned schedule with its known-depth groups captured in one hipGraph:
    # bit-identical to the direct launches, within eps of the exact resistance
    # on the stratified sample, and equal to the checker's run at the same
    # (l_b, tau) on the replay sample
    g, s, t, eps, lam, r, st, sample, cover, learned, exact = rmat22_run
    (rd, std), (rg, stg) = learned["direct"], learned["graph"]
    assert np.array_equal(rd, rg)
    for f in std.dtype.names:
        assert np.array_equal(std[f], stg[f]), f
    print(f"[graph] rmat22 learned: fallback {std['fallback'].mean():.4f}, mean l_b {std['ell_b'].mean():.2f}",
          flush=True)
    idx = np.concatenate([sample, cover])
    ex = np.array([exact[i] for i in idx.tolist()])
    fails = np.abs(rg[idx] - ex) > eps[idx]
    print(f"[coverage] rmat22 learned: {len(idx) - fails.sum()}/{len(idx)} within eps", flush=True)
    assert fails.sum() <= 0.01 * len(idx)
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s[sample], t[sample], eps[sample], lam, seed=3303,
                          schedule="fixed", fixed_lb=stg["ell_b"][sample], qid=sample,
                          tau_per_pair=stg["tau"][sample])
    parity.compare(g, s[sample], t[sample], eps[sample], lam, stg[sample], sto, tau=None,
                   tau_per_pair=stg["tau"][sample], seed=3303, qid=sample, label="rmat22 learned graph")


# ---------------------------------------------------------------------------
# learned checkpoint on a fresh Chung-Lu n = 2 * 10^6 graph
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def cl2m_run():
    g = I.chung_lu(2_000_000, 2.1, 20, 1004)
    s, t = I.uniform_pairs(g.n, 50_000, 2004)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx) as gg:
        lam = G.geer_graph_compute_lambda(gg.handle, 400, 1e-8, 7)
        ts, tt = I.uniform_pairs(g.n, 1024, 2104)
        G.geer_autotune(gg.handle, ts, tt, 0.05)
        model = G.Model(path=os.path.join(ROOT, "paper_2312_06123_amd", "data", "scheduler.geermlp"))
        p = G.geer_params_default(seed=3004, schedule=G.GEER_SCHEDULE_LEARNED, model=model.handle.value)
        r, st = G.geer_query(gg.handle, s, t, 0.05, p, stats=True)
    sample = np.random.default_rng(1).choice(np.arange(len(s)), 24, replace=False)
    return g, s, t, lam, r, st, sample


def test_cl2m_learned_applies_and_is_exact(cl2m_run):
    g, s, t, lam, r, st, sample = cl2m_run
    assert np.all(np.isfinite(r))
    assert (st["fallback"] == 0).mean() >= 0.5
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s[sample], t[sample], tol=1e-10)
    assert np.all(np.abs(r[sample] - ex) <= 0.05)


def test_cl2m_learned_replay(cl2m_run):
    g, s, t, lam, r, st, sample = cl2m_run
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s[sample], t[sample], 0.05, lam, seed=3004,
                          schedule="fixed", fixed_lb=st["ell_b"][sample], qid=sample,
                          tau_per_pair=st["tau"][sample])
    assert np.array_equal(sto["ell_b"], st["ell_b"][sample])
    parity.compare(g, s[sample], t[sample], 0.05, lam, st[sample], sto, tau=None,
                   tau_per_pair=st["tau"][sample], seed=3004, qid=sample, label="chung-lu 2M learned")


# ---------------------------------------------------------------------------
# R-MAT scale 24, 10^6 degree-proportional pairs, eps = 0.02
# ---------------------------------------------------------------------------

@pytest.fixture(scope="module")
def rmat24_run():
    import time

    t0 = time.time()
    g = I.rmat(24, 16, 0.57, 0.19, 0.19, 1005, progress=lambda m: print(f"[rmat24] {m}", flush=True))
    print(f"[rmat24] graph n={g.n} nnz={g.nnz} d_max={int(g.degrees().max())} "
          f"in {time.time() - t0:.0f} s", flush=True)
    nq, chunk = 1_000_000, 100_000
    s, t = I.degree_pairs(g, nq, 2005)
    r = np.full(nq, np.nan)
    st = None
    done, busy = 0, 0.0
    with G.Graph(g.n, g.row_ptr32(), g.col_idx) as gg:
        print(f"[rmat24] graph on the GPU after {time.time() - t0:.0f} s", flush=True)
        lam = G.geer_graph_compute_lambda(gg.handle, 400, 1e-8, 7)
        print(f"[rmat24] lambda={lam:.6f} after {time.time() - t0:.0f} s", flush=True)
        ts, tt = I.uniform_pairs(g.n, 1024, 2105)
        G.geer_autotune(gg.handle, ts, tt, 0.02)
        print(f"[rmat24] autotuned after {time.time() - t0:.0f} s", flush=True)
        model = G.Model(path=os.path.join(ROOT, "paper_2312_06123_amd", "data", "scheduler.geermlp"))
        while done < nq:
            hi = min(nq, done + chunk)
            p = G.geer_params_default(seed=3005, schedule=G.GEER_SCHEDULE_LEARNED,
                                      model=model.handle.value, qid_offset=done)
            c0 = time.time()
            rc, stc = G.geer_query(gg.handle, s[done:hi], t[done:hi], 0.02, p, stats=True)
            busy += time.time() - c0
            r[done:hi] = rc
            st = stc if st is None else np.concatenate([st, stc])
            done = hi
            print(f"[rmat24] {done} pairs in {busy:.1f} s ({done / busy:.0f} pairs/s)", flush=True)
    assert done == nq
    sample = np.random.default_rng(5).choice(np.arange(done), 24, replace=False)
    cover = np.setdiff1d(np.random.default_rng(6).choice(np.arange(done), 60, replace=False), sample)[:48]
    return g, s, t, lam, r, st, done, sample, cover


def test_rmat24_learned_replay(rmat24_run):
    g, s, t, lam, r, st, done, sample, cover = rmat24_run
    assert np.all(np.isfinite(r))
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s[sample], t[sample], 0.02, lam, seed=3005,
                          schedule="fixed", fixed_lb=st["ell_b"][sample], qid=sample,
                          tau_per_pair=st["tau"][sample])
    parity.compare(g, s[sample], t[sample], 0.02, lam, st[sample], sto, tau=None,
                   tau_per_pair=st["tau"][sample], seed=3005, qid=sample, label="rmat24 learned")


def test_rmat24_exact_on_sample(rmat24_run):
    g, s, t, lam, r, st, done, sample, cover = rmat24_run
    idx = np.concatenate([sample, cover])
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s[idx], t[idx], tol=1e-8)
    err = np.abs(r[idx] - ex)
    print(f"[coverage] rmat24: {int((err <= 0.02).sum())}/{len(idx)} within eps; "
          f"max |r' - r| = {err.max():.4f}", flush=True)
    assert np.all(err <= 0.02)
