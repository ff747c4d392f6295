"""Learned scheduler on the GPU against the FP64 references.

  * MLP gradient and Adam steps: GPU FP32 kernels vs the FP64 reference
    (relative 1e-4 of the largest entry);
  * BF16 inference within 2% of FP32 on each output;
  * features: exact (they are log2 of integers, evaluated in FP64, stored in FP32);
  * the learned schedule keeps the estimator's guarantee: |r' - r| <= eps on
    >= 99% of pairs, and each answer equals the checker run with the same
    per-pair (l_b, tau).
"""

import os

import numpy as np
import pytest

import oracle
from oracle import mlp as M
from paper_2312_06123_amd import inputs as I

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2312_06123_amd.geer")


def _data(n, seed):
    rng = np.random.default_rng(seed)
    X = rng.normal(0, 1, (n, M.F)).astype(np.float32)
    Y = rng.normal(0, 1, (n, M.O)).astype(np.float32)
    W = rng.random((n, M.O)).astype(np.float32)
    return X, Y, W


def test_mlp_gradient_matches_reference():
    m = G.Model(seed=3)
    p = m.get_params()
    X, Y, W = _data(40, 1)
    g_gpu = m.grad(X, Y, W).astype(np.float64)
    g_ref = M.grad(p.astype(np.float64), X.astype(np.float64), Y.astype(np.float64),
                   W.astype(np.float64))
    assert np.max(np.abs(g_gpu - g_ref)) <= 1e-4 * np.max(np.abs(g_ref))


def test_mlp_adam_steps_match_reference():
    m = G.Model(seed=5)
    p = m.get_params().astype(np.float64)
    X, Y, W = _data(100, 2)
    steps, B = 4, 32
    order = np.random.default_rng(3).integers(0, 100, steps * B)
    m.train(X, Y, W, steps, B, 1e-2, order=order)
    mom = np.zeros(M.P)
    vel = np.zeros(M.P)
    for k in range(steps):
        idx = order[k * B:(k + 1) * B]
        g = M.grad(p, X[idx].astype(np.float64), Y[idx].astype(np.float64), W[idx].astype(np.float64))
        p, mom, vel = M.adam_step(p, mom, vel, g, k + 1, 1e-2)
    got = m.get_params().astype(np.float64)
    assert np.max(np.abs(got - p)) <= 1e-4 * np.max(np.abs(p))


def test_mlp_forward_fp32_and_bf16():
    m = G.Model(seed=9)
    p = m.get_params().astype(np.float64)
    X, _, _ = _data(300, 4)
    ref = M.forward(p, X.astype(np.float64))
    y32 = m.forward(X, bf16=False)
    y16 = m.forward(X, bf16=True)
    scale = np.max(np.abs(ref), axis=0)
    assert np.all(np.max(np.abs(y32 - ref), axis=0) <= 1e-5 * scale)
    assert np.all(np.max(np.abs(y16 - ref), axis=0) <= 2e-2 * scale)


def test_mlp_training_reduces_loss_and_checkpoint_roundtrip(tmp_path):
    rng = np.random.default_rng(6)
    X = rng.normal(0, 1, (2000, M.F)).astype(np.float32)
    Y = np.stack([X[:, 0] * 2 + X[:, 1], np.abs(X[:, 2]), X[:, 3] * X[:, 4]], axis=1).astype(np.float32)
    W = np.ones_like(Y)
    m = G.Model(seed=1)
    loss = m.train(X, Y, W, 1500, 64, 3e-3)
    assert loss[-100:].mean() < 0.2 * loss[:20].mean()
    path = str(tmp_path / "m.geermlp")
    m.save(path)
    m2 = G.Model(path=path)
    assert np.array_equal(m.get_params(), m2.get_params())
    assert np.array_equal(m.forward(X[:50]), m2.forward(X[:50]))
    # training resumes from the checkpoint exactly as it would have continued
    l_a = m.train(X, Y, W, 50, 64, 1e-3)
    l_b = m2.train(X, Y, W, 50, 64, 1e-3)
    assert np.array_equal(l_a, l_b) and np.array_equal(m.get_params(), m2.get_params())


def snap(r):
    """log2 of a cost ratio as stored: rounded to the nearest half."""
    return np.round(2.0 * np.log2(r)) / 2.0


def test_features_match_definition():
    g = I.chung_lu(5000, 2.1, 10, 71)
    lam = oracle.lambda_arpack(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 200, 72)
    s[:20], t[:20] = I.edge_pairs(g, 20, 73)
    deg = g.degrees()
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        G.geer_graph_set_costs(gg.handle, 5.0, 3e5)
        f = G.geer_features(gg.handle, s, t, 0.05)
    def log_psi1(i):
        # Eq. (Delta-st) after one product from the checker's hop-1 vectors
        ell = oracle.ell(deg[s[i]], deg[t[i]], 0.05, lam)
        if ell <= 1:
            return np.log2(2.0 ** -40 / 0.05)
        x, y, _, _, _ = oracle.smm_vectors(g.row_ptr, g.col_idx, int(s[i]), int(t[i]), 1)
        psi = oracle.psi(ell - 1, *oracle.top2(x), *oracle.top2(y), float(deg[s[i]]), float(deg[t[i]]))
        return np.log2(psi / 0.05)

    for i in range(len(s)):
        ns = g.col_idx[g.row_ptr[s[i]]:g.row_ptr[s[i] + 1]]
        nt = g.col_idx[g.row_ptr[t[i]]:g.row_ptr[t[i] + 1]]
        want = [np.log2(deg[s[i]]), np.log2(deg[t[i]]),
                oracle.ell(deg[s[i]], deg[t[i]], 0.05, lam) / 16.0,
                np.log2(1 + deg[ns].sum()), np.log2(1 + deg[nt].sum()),
                np.log2(deg[ns].min()), np.log2(deg[nt].min()),
                float(t[i] in ns), np.log2(1 + len(np.intersect1d(ns, nt))),
                np.log2(1 / (1 - lam)), np.log2(0.05), snap(5.0), snap(3e5), log_psi1(i)]
        assert np.allclose(f[i], np.array(want, dtype=np.float32), rtol=1e-6, atol=1e-6), i


def _trained_model(gg, g, lam):
    """A small model trained on this graph's own sweeps (fast)."""
    from paper_2312_06123_amd import scheduler as S

    s, t = I.uniform_pairs(g.n, 300, 81)
    runs = S.sweep(gg, s, t, 0.1)
    r_ref = S.reference(gg, s, t)
    feats = G.geer_features(gg.handle, s, t, 0.1)
    X, Y, W = S.label(feats, runs, r_ref, np.random.default_rng(0), n_rho=2)
    m, losses, _ = S.train_model(X, Y, W, steps=800)
    assert losses[-50:].mean() < losses[:50].mean()
    return m


def test_learned_schedule_guarantee_and_replay():
    g = I.chung_lu(20000, 2.1, 20, 102)
    lam = oracle.lambda_arpack(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 400, 82)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        m = _trained_model(gg, g, lam)
        p = G.geer_params_default(seed=17, schedule=G.GEER_SCHEDULE_LEARNED, model=m.handle.value)
        r, st = G.geer_query(gg.handle, s, t, 0.1, p, stats=True)
    ex, _ = oracle.exact_cg(g.row_ptr, g.col_idx, s, t)
    assert np.mean(np.abs(r - ex) <= 0.1) >= 0.99
    assert np.all((st["ell_b"] >= 0) & (st["ell_b"] <= st["ell"]))
    assert np.all((st["tau"] >= 1) & (st["tau"] <= 8))
    learned = st["fallback"] == 0
    assert learned.mean() > 0.5
    # replay the learned pairs with the checker at the same (l_b, tau)
    idx = np.flatnonzero(learned)
    ro, sto = oracle.geer(g.row_ptr, g.col_idx, s[idx], t[idx], 0.1, lam, seed=17,
                          schedule="fixed", fixed_lb=st["ell_b"][idx], qid=idx,
                          tau_per_pair=st["tau"][idx])
    assert np.array_equal(sto["ell_b"], st["ell_b"][idx])
    same = (sto["eta1"] == st["eta1"][idx]) & (sto["batches_run"] == st["batches_run"][idx])
    assert same.mean() >= 0.95
    assert np.all(np.abs(r[idx][same] - ro[same]) <= 1e-5 * np.maximum(1.0, np.abs(ro[same])))


def test_learned_answers_stable_under_cost_noise():
    # The cost ratios come from timings; stored on a sqrt(2) grid, a +-5%
    # change of either ratio leaves the learned schedule and every answer
    # bit-identical (the shipped checkpoint, a graph it was not trained on).
    g = I.chung_lu(20000, 2.1, 20, 102)
    lam = oracle.lambda_arpack(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 600, 83)
    path = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                        "paper_2312_06123_amd", "data", "scheduler.geermlp")
    out = []
    m = G.Model(path=path)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        for f2, fd in ((1.0, 1.0), (1.05, 0.95), (0.95, 1.05), (1.05, 1.05), (0.95, 0.95)):
            G.geer_graph_set_costs(gg.handle, 16.0 * f2, 2.0 ** 20 * fd)
            feats = G.geer_features(gg.handle, s[:4], t[:4], 0.05)
            assert np.all(feats[:, 11] == 4.0) and np.all(feats[:, 12] == 20.0)
            p = G.geer_params_default(seed=19, schedule=G.GEER_SCHEDULE_LEARNED, model=m.handle.value)
            out.append(G.geer_query(gg.handle, s, t, 0.05, p, stats=True))
    m.close()
    r0, st0 = out[0]
    assert (st0["fallback"] == 0).mean() > 0.5
    for r, st in out[1:]:
        assert np.array_equal(r, r0)
        for f in st0.dtype.names:
            assert np.array_equal(st[f], st0[f]), f
