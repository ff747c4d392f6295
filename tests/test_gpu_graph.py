"""Captured launches (GEER_FLAG_GRAPH_LAUNCH) against direct launches.

Every answer and every field of every record must be bit-identical: the
captured graph runs the same kernels on the same data, and no result depends
on the walk grid (a chunk's partial is the same whichever wave walks it) or on
the column tile.  Covered: FIXED depths over several groups on two slot sets
(capture, replay, capture again after the inputs change), FP64 vectors, the
device entry point, LEARNED (the shipped checkpoint, and untrained weights
with a narrow feature range so that many pairs fall back to the greedy
switch, whose groups are launched directly after the graph), the clean
GEER_E_OOM of a captured round beyond the reserved chunk partials, while
direct launches of the same call (chunk bounds read per group) answer it.
"""

import os

import numpy as np
import pytest

import oracle
from paper_2312_06123_amd import inputs as I

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2312_06123_amd.geer")
ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def cl_graph():
    g = I.chung_lu(20000, 2.1, 20, 102)
    lam = oracle.lambda_arpack(g.row_ptr, g.col_idx)
    return g, lam


def _same(a, b):
    (r1, s1), (r2, s2) = a, b
    assert np.array_equal(r1, r2)
    for f in s1.dtype.names:
        assert np.array_equal(s1[f], s2[f]), f


def _run(gg, s, t, eps, graph, **kw):
    flags = kw.pop("flags", 0) | (G.GEER_FLAG_GRAPH_LAUNCH if graph else 0)
    p = G.geer_params_default(flags=flags, **kw)
    return G.geer_query(gg.handle, s, t, eps, p, stats=True)


@pytest.mark.parametrize("fp64", [False, True])
def test_graph_fixed_depths_identical(cl_graph, fp64):
    g, lam = cl_graph
    rng = np.random.default_rng(3)
    s, t = I.uniform_pairs(g.n, 700, 51)
    s[:40], t[:40] = I.edge_pairs(g, 40, 52)
    depth = rng.integers(0, 5, len(s)).astype(np.int32)
    depth2 = rng.integers(0, 5, len(s)).astype(np.int32)
    fl = G.GEER_FLAG_FP64_VECTORS if fp64 else 0
    # 11 batches in groups of 3: four groups alternating over two slot sets
    kw = dict(seed=41, schedule=G.GEER_SCHEDULE_FIXED, group_batches=3, flags=fl)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        eager = _run(gg, s, t, 0.1, False, fixed_ell_b=depth.ctypes.data, **kw)
        G.geer_profile_enable(gg.handle, True)
        first = _run(gg, s, t, 0.1, True, fixed_ell_b=depth.ctypes.data, **kw)
        replay = _run(gg, s, t, 0.1, True, fixed_ell_b=depth.ctypes.data, **kw)
        prof = G.geer_profile_read(gg.handle)
        G.geer_profile_enable(gg.handle, False)
        assert prof["graph"]["launches"] == 2
        assert prof["walk"]["launches"] == 0  # every walk ran inside the graphs
        _same(eager, first)
        _same(eager, replay)
        # other depths: captured again
        eager2 = _run(gg, s, t, 0.1, False, fixed_ell_b=depth2.ctypes.data, **kw)
        again = _run(gg, s, t, 0.1, True, fixed_ell_b=depth2.ctypes.data, **kw)
        _same(eager2, again)
        assert not np.array_equal(eager[1]["ell_b"], eager2[1]["ell_b"])


def _model(kind):
    if kind == "shipped":
        return G.Model(path=os.path.join(ROOT, "paper_2312_06123_amd", "data", "scheduler.geermlp"))
    # untrained weights; pairs with d(s) above ~2^3.3 leave the (narrow)
    # range of feature 0 and fall back to the greedy switch
    m = G.Model(seed=7)
    F = G.MLP_FEATURES
    lo, hi = np.full(F, -100.0), np.full(F, 100.0)
    lo[0], hi[0] = 0.0, 3.0
    m.set_norm(np.zeros(F), np.full(F, 4.0), lo, hi)
    return m


@pytest.mark.parametrize("kind", ["shipped", "fallback"])
def test_graph_learned_and_device_entry(cl_graph, kind):
    torch = pytest.importorskip("torch")
    g, lam = cl_graph
    s, t = I.uniform_pairs(g.n, 900, 53)
    s[:60], t[:60] = I.edge_pairs(g, 60, 54)
    eps = np.random.default_rng(4).choice(np.array([0.03, 0.05, 0.1]), len(s))
    model = _model(kind)
    kw = dict(seed=43, schedule=G.GEER_SCHEDULE_LEARNED, model=model.handle.value, group_batches=4)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        G.geer_graph_set_costs(gg.handle, 16.0, 2.0 ** 20)
        eager = _run(gg, s, t, eps, False, **kw)
        graph = _run(gg, s, t, eps, True, **kw)
        _same(eager, graph)
        fb = eager[1]["fallback"]
        print(f"[graph] learned ({kind}): {int(fb.sum())} of {len(s)} pairs fall back", flush=True)
        if kind == "fallback":
            # greedy groups launched after the graph, static ones inside it
            assert 0 < fb.sum() < len(s) - 256
        # the device entry point: capture, then replay
        ds = torch.from_numpy(s).cuda()
        dt = torch.from_numpy(t).cuda()
        de = torch.from_numpy(eps).cuda()
        for _ in range(2):
            dr = torch.full((len(s),), float("nan"), dtype=torch.float64, device="cuda")
            p = G.geer_params_default(flags=G.GEER_FLAG_GRAPH_LAUNCH, **kw)
            G.geer_query_device(gg.handle, ds, dt, de, dr, p)
            torch.cuda.synchronize()
            assert np.array_equal(dr.cpu().numpy(), eager[0])
    model.close()


def test_graph_round_beyond_reserved_partials_is_clean_oom():
    g = I.erdos_renyi_path(2000, 10, 101)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 64, 55)
    eps, tau, delta = 2e-4, 5, 0.01
    deg = g.degrees()
    # the checker's FP64 schedule quantities at depth 1: the group's first
    # round already needs more chunk partials than the 2^24 reserved, while
    # no single batch reaches 2^32 walk pairs (that is another error)
    chunks, largest = 0, 0
    for j in range(len(s)):
        x, y, _, _, _ = oracle.smm_vectors(g.row_ptr, g.col_idx, int(s[j]), int(t[j]), 1)
        lf = oracle.ell(deg[s[j]], deg[t[j]], eps, lam) - 1
        psi = oracle.psi(lf, *oracle.top2(x), *oracle.top2(y), float(deg[s[j]]), float(deg[t[j]]))
        eta1 = int(np.ceil(oracle.eta_star(psi, eps, tau, delta) / 2 ** (tau - 1)))
        chunks += -(-eta1 // 32)
        largest = max(largest, eta1 << (tau - 1))
    assert chunks > 2 * 2 ** 24 and largest < 2 ** 31
    depth = np.ones(len(s), dtype=np.int32)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        with pytest.raises(G.GeerError) as e:
            _run(gg, s, t, eps, True, seed=1, schedule=G.GEER_SCHEDULE_FIXED, fixed_ell_b=depth.ctypes.data)
        assert e.value.status == G.GEER_E_OOM
        # the library is usable again, captured or not
        kw = dict(seed=2, schedule=G.GEER_SCHEDULE_FIXED, fixed_ell_b=depth.ctypes.data)
        _same(_run(gg, s, t, 0.1, False, **kw), _run(gg, s, t, 0.1, True, **kw))


def test_graph_buffers_return_to_the_device(cl_graph):
    # Captures with the handle's own fork/join events after an earlier capture
    # left the buffers their graph addressed unreturnable when freed; the
    # library captures with fresh events.  Two captures (the slot buffers'
    # state changes after the first call), a replay, then the handle is
    # destroyed: the device's free memory is back where it was.
    torch = pytest.importorskip("torch")
    g, lam = cl_graph
    s, t = I.uniform_pairs(g.n, 700, 56)
    depth = np.random.default_rng(5).integers(1, 5, len(s)).astype(np.int32)
    torch.cuda.synchronize()
    free0 = torch.cuda.mem_get_info()[0]
    kw = dict(seed=44, schedule=G.GEER_SCHEDULE_FIXED, group_batches=3, fixed_ell_b=depth.ctypes.data)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        for _ in range(3):
            _run(gg, s, t, 0.1, True, **kw)
        torch.cuda.synchronize()
        used = free0 - torch.cuda.mem_get_info()[0]
    torch.cuda.synchronize()
    back = torch.cuda.mem_get_info()[0]
    print(f"[graph] buffers {used / 1e9:.2f} GB; not returned {(free0 - back) / 1e9:.3f} GB", flush=True)
    assert used > 256 << 20
    assert free0 - back < 64 << 20


def test_direct_launches_not_limited_by_reserved_partials():
    # A captured plan reserves a fixed number of chunk partials; direct
    # launches read each group's chunk bound and size the partials to it, so
    # a call whose first round does not fit the captured plan still answers
    # within eps.
    g = I.erdos_renyi_path(2000, 10, 101)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 64, 57)
    eps, tau, delta = 6e-4, 2, 0.01
    deg = g.degrees()
    chunks = 0
    for j in range(len(s)):
        x, y, _, _, _ = oracle.smm_vectors(g.row_ptr, g.col_idx, int(s[j]), int(t[j]), 1)
        lf = oracle.ell(deg[s[j]], deg[t[j]], eps, lam) - 1
        psi = oracle.psi(lf, *oracle.top2(x), *oracle.top2(y), float(deg[s[j]]), float(deg[t[j]]))
        chunks += -(-int(np.ceil(oracle.eta_star(psi, eps, tau, delta) / 2 ** (tau - 1))) // 32)
    assert chunks > 2 ** 24  # the first round does not fit the fixed plan
    depth = np.ones(len(s), dtype=np.int32)
    kw = dict(seed=3, schedule=G.GEER_SCHEDULE_FIXED, fixed_ell_b=depth.ctypes.data, tau=tau, delta=delta)
    exact = oracle.exact_pinv(g.row_ptr, g.col_idx, s, t)
    with G.Graph(g.n, g.row_ptr32(), g.col_idx, lam=lam) as gg:
        with pytest.raises(G.GeerError) as e:
            _run(gg, s, t, eps, True, **kw)
        assert e.value.status == G.GEER_E_OOM
        r, st = _run(gg, s, t, eps, False, **kw)
        err = np.abs(r - exact)
        print(f"[graph] rerun with bounds: max |err| {err.max():.2e} (eps {eps})", flush=True)
        assert np.all(err <= eps)
        assert np.all(st["ell_b"] == 1)
        assert np.all(st["walk_pairs"] > 0)
