"""CPU checks of the learned scheduler's labelling rule.

Each training pair is labelled with the fixed schedule (l_b, tau) of least
cost, where cost = walk steps * (rho_v if the steps read vector values else 1)
+ rho2 * (hop-2 work) * [l_b >= 2] + rhod * max(l_b - 2, 0), under cost
ratios rho2, rhod drawn per sample; the labels are the schedule's effective
depth, its tau and the log error of its answer.  Steps read vector values at
l_b >= 2, and at l_b = 1 when a row of s or t is longer than 256 entries.
These tests feed hand-made sweep results whose cheapest schedule is known.
"""

import numpy as np
import pytest

G = pytest.importorskip("paper_2312_06123_amd.geer")
S = pytest.importorskip("paper_2312_06123_amd.scheduler")


def _stats(n, ell, ell_b, walk_pairs):
    st = np.zeros(n, dtype=G.STATS_DTYPE)
    st["ell"] = ell
    st["ell_b"] = ell_b
    st["walk_pairs"] = walk_pairs
    return st


def _runs(n, table):
    """table: (l_b, tau) -> walk pairs per pair (arrays); l = 10 for all."""
    return {key: (np.full(n, 1.0), _stats(n, 10, key[0], wp)) for key, wp in table.items()}


def _feats(n, work2):
    x = np.zeros((n, G.MLP_FEATURES), dtype=np.float32)
    x[:, 3] = np.log2(1.0 + work2 / 2.0)  # neighbour-degree sums of s and t (half each)
    x[:, 4] = np.log2(1.0 + work2 / 2.0)
    return x


def test_label_picks_cheapest_schedule_and_sets_cost_features():
    n = 3
    # pair 0: shallow is far cheaper in walks; pair 1: depth 2 saves many walks;
    # pair 2: depth 3 saves a few walks more than depth 2
    table = {
        (1, 2): np.array([10.0, 1e6, 1e6]),
        (2, 2): np.array([1e6, 10.0, 1e4]),
        (3, 2): np.array([1e6, 1e6, 9.0e3]),
    }
    runs = _runs(n, table)
    feats = _feats(n, np.array([100.0, 100.0, 100.0]))
    r_ref = np.full(n, 1.0)
    X, Y, W = S.label(feats, runs, r_ref, np.random.default_rng(0), n_rho=4)
    assert X.shape == (4 * n, G.MLP_FEATURES) and Y.shape == (4 * n, 3) and W.shape == (4 * n, 3)
    for k in range(4):
        x, y = X[k * n:(k + 1) * n], Y[k * n:(k + 1) * n]
        rho2, rhod = 2.0 ** x[:, 11], 2.0 ** x[:, 12]
        for i in range(n):
            costs = {key: 2.0 * table[key][i] * (10 - key[0]) * (S.RHO_V if key[0] >= 2 else 1.0)
                     + rho2[i] * 100.0 * (key[0] >= 2) + rhod[i] * max(key[0] - 2, 0) for key in table}
            best = min(costs, key=costs.get)
            assert y[i, 0] == best[0] and y[i, 1] == best[1]
        assert np.all(y[:, 2] == np.float32(np.log10(1e-6)))  # answers equal r_ref
    # pair 0 always stays shallow, pair 1 always takes depth 2
    assert np.all(Y[0::n, 0] == 1) and np.all(Y[1::n, 0] == 2)


def test_label_uses_effective_depth_and_error():
    # a schedule asked for depth 3 that stopped at l = 2 is labelled with 2;
    # the error label is log10 |r' - r_ref| (+1e-6)
    n = 1
    runs = {(3, 5): (np.array([1.5]), _stats(n, 2, 2, np.array([0.0])))}
    X, Y, W = S.label(_feats(n, np.array([10.0])), runs, np.array([1.0]), np.random.default_rng(1),
                      n_rho=1)
    assert Y[0, 0] == 2 and Y[0, 1] == 5
    assert Y[0, 2] == pytest.approx(np.log10(0.5 + 1e-6), rel=1e-6)
    assert np.allclose(W, [[1.0, 0.25, 0.5]])


@pytest.mark.parametrize("rho_v", [1.0, 2.0, 3.0])
def test_label_weights_steps_that_read_vectors(rho_v):
    # two pairs with the same sweep; pair 0's rows are short (its depth-1 walks
    # evaluate the one-hop vectors from the graph), pair 1's row of s has 300
    # entries (its depth-1 walks read vector values, as all depth-2 walks do)
    n = 2
    table = {(1, 2): np.array([100.0, 100.0]), (2, 2): np.array([60.0, 60.0])}
    runs = _runs(n, table)
    feats = _feats(n, np.array([0.0, 0.0]))
    feats[:, 0] = np.log2([2.0, 300.0])
    feats[:, 1] = np.log2([3.0, 5.0])
    X, Y, W = S.label(feats, runs, np.full(n, 1.0), np.random.default_rng(2), n_rho=2, rho_v=rho_v)
    # steps at depth 1: 2 * 100 * 9 = 1800; at depth 2: 2 * 60 * 8 = 960
    c1 = [1800.0, 1800.0 * rho_v]
    c2 = 960.0 * rho_v
    for i in range(n):
        assert np.all(Y[i::n, 0] == (2 if c2 < c1[i] else 1)), i
    if rho_v == 2.0:
        assert np.all(Y[0::n, 0] == 1) and np.all(Y[1::n, 0] == 2)
