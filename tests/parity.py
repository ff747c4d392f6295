"""Pair-by-pair comparison of the library's per-query records with the checker's.

Every pair is compared, not only the pairs whose schedules agree:

  * l (Eq. ell) exactly;
  * at the SMM depth l_b the library ran: r_b, psi (Eq. Delta-st) and eta*
    (Eq. etas-star) against the checker's FP64 values at that depth;
  * where the checker's own schedule took another decision, the quantity
    that decided it, computed by the checker alone, must lie within FP32
    rounding of its threshold: the support degree sum against h(l - l_b) for
    the greedy switch (Eq. smm-amc), eta*/2^(tau-1) against an integer for
    eta_1, and the Bernstein width f (Eq. fx) against eps/2 for the batch
    that stopped on one side only;
  * where every decision agrees: walk pairs exactly and r' to the vector
    precision.

Only checker functions compute the reference side; the library's depth is
used to pick which hop the checker's vectors are taken at.
"""

from __future__ import annotations

import math

import numpy as np

import oracle

# FP32 vectors: one rounding per stored entry plus the accumulated rounding
# of l_b products, well below 1e-6 relative for r_b and psi; eta* carries
# psi^2, twice its relative error.
TOL32 = {"rb": 1e-6, "psi": 1e-6, "eta": 2e-6, "r": 1e-5}
TOL64 = {"rb": 1e-12, "psi": 1e-12, "eta": 2e-12, "r": 1e-9}
# half-width of the band around a threshold inside which FP32 inputs may
# decide either way (relative)
BAND32 = 1e-5
BAND64 = 1e-11
# Bernstein width: f depends on the empirical variance, in which the FP32
# rounding of the summed values can cancel; the band is wider
BAND_F32 = 1e-3
BAND_F64 = 1e-9


def _rel(a: float, b: float) -> float:
    if a == b:
        return 0.0
    return abs(a - b) / max(abs(b), 1e-300)


def _ceil_band(a: float, band: float) -> tuple[int, int]:
    return math.ceil(a * (1.0 - band)), math.ceil(a * (1.0 + band))


def compare(g, s, t, eps, lam, st, sto, *, tau, delta=0.01, seed=0, qid=None, tau_per_pair=None,
            fp64=False, label=""):
    """Assert the checks above for every pair; return the counts of each case."""
    tol = TOL64 if fp64 else TOL32
    band = BAND64 if fp64 else BAND32
    band_f = BAND_F64 if fp64 else BAND_F32
    deg = g.degrees()
    n = len(s)
    eps = np.broadcast_to(np.asarray(eps, dtype=np.float64), (n,))
    qid = np.arange(n) if qid is None else np.asarray(qid)
    counts = {"pairs": n, "agree": 0, "depth_tie": 0, "eta1_tie": 0, "batch_tie": 0}
    vec_cache = {}

    def vectors(j, hops):
        key = (j, hops)
        if key not in vec_cache:
            vec_cache[key] = oracle.smm_vectors(g.row_ptr, g.col_idx, int(s[j]), int(t[j]), int(hops))
        return vec_cache[key]

    for j in range(n):
        where = f"{label} pair {j} (s={s[j]}, t={t[j]}, eps={eps[j]})"
        l = int(sto["ell"][j])
        assert int(st["ell"][j]) == l, where
        if s[j] == t[j]:
            assert st["r_b"][j] == 0.0 and st["walk_pairs"][j] == 0, where
            counts["agree"] += 1
            continue
        tq = int(tau_per_pair[j]) if tau_per_pair is not None else int(tau)
        e = float(eps[j])
        ds, dt = float(deg[s[j]]), float(deg[t[j]])
        lb_g, lb_o = int(st["ell_b"][j]), int(sto["ell_b"][j])
        if lb_g == lb_o:
            rb_o, psi_o, es_o = float(sto["r_b"][j]), float(sto["psi"][j]), float(sto["eta_star"][j])
        else:
            # greedy switch: at the first hop where the two differ, one side
            # stopped and the other did not
            h0 = min(lb_g, lb_o)
            x, y, sx, sy, _ = vectors(j, h0)
            supp = int(deg[sx].sum() + deg[sy].sum())
            psi_h = oracle.psi(l - h0, *oracle.top2(x), *oracle.top2(y), ds, dt)
            a = oracle.eta_star(psi_h, e, tq, delta) / 2.0 ** (tq - 1)
            lo, hi = _ceil_band(a, band)
            w = 2.0 ** tq - 1.0
            assert (supp > w * lo) != (supp > w * hi), (
                f"{where}: depths {lb_g} vs {lb_o} but the switch rule at hop {h0} is not a tie "
                f"(supp {supp}, h {w * math.ceil(a)})")
            x, y, _, _, rb_o = vectors(j, lb_g)
            if l > lb_g:
                psi_o = oracle.psi(l - lb_g, *oracle.top2(x), *oracle.top2(y), ds, dt)
                es_o = oracle.eta_star(psi_o, e, tq, delta)
            else:
                psi_o = es_o = 0.0
        assert _rel(float(st["r_b"][j]), rb_o) <= tol["rb"] or abs(st["r_b"][j] - rb_o) <= 1e-15, (
            f"{where}: r_b {st['r_b'][j]!r} vs {rb_o!r}")
        assert _rel(float(st["psi"][j]), psi_o) <= tol["psi"], f"{where}: psi {st['psi'][j]!r} vs {psi_o!r}"
        assert _rel(float(st["eta_star"][j]), es_o) <= tol["eta"], (
            f"{where}: eta* {st['eta_star'][j]!r} vs {es_o!r}")
        if lb_g != lb_o:
            counts["depth_tie"] += 1
            continue
        if int(st["eta1"][j]) != int(sto["eta1"][j]):
            a = es_o / 2.0 ** (tq - 1)
            lo, hi = _ceil_band(a, band)
            assert lo != hi, f"{where}: eta_1 {st['eta1'][j]} vs {sto['eta1'][j]}, eta*/2^(tau-1) = {a!r}"
            counts["eta1_tie"] += 1
            continue
        b_g, b_o = int(st["batches_run"][j]), int(sto["batches_run"][j])
        if b_g != b_o:
            # the first batch that stopped on one side only
            i0 = min(b_g, b_o) - 1
            x, y, _, _, _ = vectors(j, lb_o)
            count = int(sto["eta1"][j]) << i0
            z = oracle.amc_samples(g.row_ptr, g.col_idx, int(s[j]), int(t[j]), x, y, l - lb_o, seed,
                                   int(qid[j]), i0, count)
            zm = z.sum() / count
            var = max(0.0, (z * z).sum() / count - zm * zm)
            f = oracle.bernstein(count, var, psi_o, delta / tq)
            assert abs(f / (e / 2.0) - 1.0) <= band_f, (
                f"{where}: batches {b_g} vs {b_o}, checker's f at batch {i0 + 1} = {f!r} against eps/2")
            counts["batch_tie"] += 1
            continue
        assert int(st["walk_pairs"][j]) == int(sto["walk_pairs"][j]), where
        r_g = float(st["r_b"][j] + st["r_f"][j])
        r_o = float(sto["r"][j])
        assert abs(r_g - r_o) <= tol["r"] * max(1.0, abs(r_o)), f"{where}: r' {r_g!r} vs {r_o!r}"
        counts["agree"] += 1
    print(f"[parity] {label}: {counts}", flush=True)
    return counts
