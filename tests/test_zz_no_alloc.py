"""The allocation-free AMC entry point (geer_amc_device_noalloc) against
geer_amc on the same values: r_f and every field of the record bit-identical,
on two calls in a row (the second on a smaller graph with fewer walks), then
FP64 vectors, a repeat of the first call, and the two error paths (a batch
beyond the fixed scratch, invalid vectors) with the output left untouched.
"""

import numpy as np
import pytest

import oracle
from paper_2312_06123_amd import inputs as I

pytestmark = pytest.mark.gpu

G = pytest.importorskip("paper_2312_06123_amd.geer")
torch = pytest.importorskip("torch")

SCRATCH_BYTES = 16 << 20
ZPART_CAP = (SCRATCH_BYTES - 16384) // 16  # chunk partials the fixed scratch holds


def _vectors(g, s, t, hops, fp64):
    x, y, _, _, _ = oracle.smm_vectors(g.row_ptr, g.col_idx, s, t, hops)
    dt = np.float64 if fp64 else np.float32
    return x.astype(dt), y.astype(dt)


def _noalloc(gg, s, t, x, y, eps, lf, seed, q, fp64):
    xy = torch.from_numpy(np.stack([x, y], axis=1).reshape(-1).copy()).cuda()
    d_rf = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
    d_st = torch.zeros(G.STATS_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    G.geer_amc_device_noalloc(gg.handle, s, t, xy.data_ptr(), eps, lf, d_rf.data_ptr(),
                              d_st.data_ptr(), seed=seed, q=q, fp64=fp64)
    torch.cuda.synchronize()
    st = np.frombuffer(d_st.cpu().numpy().tobytes(), dtype=G.STATS_DTYPE)[0]
    return float(d_rf.cpu().numpy()[0]), st


def _same(gg, g, s, t, hops, lf, eps, seed, q, fp64):
    x, y = _vectors(g, s, t, hops, fp64)
    rf_ref, st_ref = G.geer_amc(gg.handle, s, t, x.astype(np.float64), y.astype(np.float64), eps, lf,
                                seed=seed, q=q, fp64=fp64)
    rf, st = _noalloc(gg, s, t, x, y, eps, lf, seed, q, fp64)
    assert st_ref["walk_pairs"] > 0
    assert rf == rf_ref, (rf, rf_ref)
    for f in G.STATS_DTYPE.names:
        assert st[f] == st_ref[f], (f, st[f], st_ref[f])
    return rf


def test_noalloc_amc_matches_allocating_entry_point():
    big = I.chung_lu(20000, 2.1, 20, 102)
    small = I.erdos_renyi_path(2000, 10, 101)
    with G.Graph(big.n, big.row_ptr32(), big.col_idx) as gb, \
            G.Graph(small.n, small.row_ptr32(), small.col_idx) as gs:
        r1 = _same(gb, big, 0, 17, 2, 8, 0.05, seed=5, q=3, fp64=False)
        # second call, smaller input: a smaller graph, fewer hops and walks
        _same(gs, small, 4, 900, 1, 5, 0.1, seed=6, q=1, fp64=False)
        _same(gs, small, 11, 1500, 2, 6, 0.1, seed=7, q=2, fp64=True)
        # the shared scratch keeps nothing from the calls in between
        assert _same(gb, big, 0, 17, 2, 8, 0.05, seed=5, q=3, fp64=False) == r1


def test_noalloc_amc_rejects_batches_beyond_scratch_and_bad_vectors():
    g = I.erdos_renyi_path(2000, 10, 101)
    s, t, hops, lf, tau, delta = 4, 900, 1, 5, 5, 0.01
    x, y = _vectors(g, s, t, hops, False)
    deg = g.degrees()
    psi = oracle.psi(lf, *oracle.top2(x.astype(np.float64)), *oracle.top2(y.astype(np.float64)),
                     float(deg[s]), float(deg[t]))
    # eps for eta* = 2e8 walk pairs: the last batch needs ~6e6 chunks of 32
    # pairs, beyond the scratch but below the 2^32-pair limit of a batch
    eps = float(np.sqrt(2.0 * psi * psi * np.log(2.0 * tau / delta) / 2e8))
    eta1 = int(np.ceil(oracle.eta_star(psi, eps, tau, delta) / 2 ** (tau - 1)))
    chunks = -(-(eta1 << (tau - 1)) // 32)
    assert ZPART_CAP < chunks and (eta1 << (tau - 1)) < 2 ** 32
    with G.Graph(g.n, g.row_ptr32(), g.col_idx) as gg:
        with pytest.raises(G.GeerError) as e:
            _noalloc(gg, s, t, x, y, eps, lf, 0, 0, False)
        assert e.value.status == G.GEER_E_OOM
        xy = torch.from_numpy(np.stack([x, y], axis=1).reshape(-1).copy()).cuda()
        xy[7] = -1.0
        d_rf = torch.full((1,), float("nan"), dtype=torch.float64, device="cuda")
        with pytest.raises(G.GeerError) as e:
            G.geer_amc_device_noalloc(gg.handle, s, t, xy.data_ptr(), 0.1, lf, d_rf.data_ptr())
        assert e.value.status == G.GEER_E_INVALID_ARG
        torch.cuda.synchronize()
        assert np.isnan(d_rf.cpu().numpy()[0])
        # the entry point still works after the failed calls
        _same(gg, g, s, t, hops, lf, 0.1, seed=8, q=0, fp64=False)
