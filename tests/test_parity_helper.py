"""CPU checks of the pair-by-pair comparison used by the GPU parity tests:
the checker compared with itself passes, and records that differ from the
checker's in a way that no FP32 tie explains are rejected."""

import numpy as np
import pytest

import oracle
import parity
from paper_2312_06123_amd import inputs as I

GPU_FIELDS = ["ell", "ell_b", "tau", "batches_run", "eta1", "walk_pairs", "supp_sum", "r_b", "r_f",
              "psi", "eta_star"]


def _as_library_records(sto, tau):
    dt = np.dtype([(f, np.float64 if f in ("r_b", "r_f", "psi", "eta_star") else np.int64)
                   for f in GPU_FIELDS])
    st = np.zeros(len(sto), dtype=dt)
    for f in GPU_FIELDS:
        st[f] = tau if f == "tau" else sto[f]
    return st


@pytest.fixture(scope="module")
def run():
    g = I.chung_lu(800, 2.1, 8, 71)
    lam = oracle.lambda_dense(g.row_ptr, g.col_idx)
    s, t = I.uniform_pairs(g.n, 80, 72)
    s[0] = t[0]
    _, sto = oracle.geer(g.row_ptr, g.col_idx, s, t, 0.05, lam, seed=4)
    return g, lam, s, t, sto


def test_checker_against_itself_agrees(run):
    g, lam, s, t, sto = run
    cnt = parity.compare(g, s, t, 0.05, lam, _as_library_records(sto, 5), sto, tau=5, seed=4,
                         fp64=True, label="self")
    assert cnt["agree"] == len(s)


@pytest.mark.parametrize("field,delta", [("ell", 1), ("ell_b", 1), ("eta1", 1), ("batches_run", 1),
                                         ("walk_pairs", 1), ("r_b", 1e-4), ("psi", 1e-4),
                                         ("r_f", 1e-3)])
def test_unexplained_difference_is_rejected(run, field, delta):
    g, lam, s, t, sto = run
    st = _as_library_records(sto, 5)
    j = int(np.flatnonzero((sto["ell_b"] >= 1) & (sto["ell_b"] < sto["ell"]) &
                           (sto["batches_run"] >= 1) & (sto["batches_run"] < 5))[0])
    st[field][j] = st[field][j] + delta
    with pytest.raises(AssertionError):
        parity.compare(g, s, t, 0.05, lam, st, sto, tau=5, seed=4, fp64=True, label="planted")
