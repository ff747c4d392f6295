"""CPU FP64 checker for GEER (Yang & Tang, pairwise effective resistance).

TEST INFRASTRUCTURE ONLY.  This package is the plain, slow reference the GPU
library is checked against.  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product path never does.  It
shares no code with the GPU library and does not import it.

Parts:
  * ``geer_oracle.c`` (built into ``liboracle.so``): Philox4x32-10, one SMM
    product, the scalar formulas (Eqs. ell, Delta-st, etas-star, fx, the walk
    budget h), walk traces, Algorithm AMC, Algorithm GEER with the greedy
    switch of Eq. (smm-amc) or a fixed depth, the truncated series of
    Eq. (r-ell), and Jacobi-PCG for the exact resistance of Definition 2.1.
  * ``mlp``: FP64 reference of the learned scheduler's network, its
    gradients and the Adam update.
  * numpy/LAPACK: the exact resistance from the Laplacian pseudo-inverse
    (Definition 2.1) for small graphs, and lambda = max(|lambda_2|, |lambda_n|)
    of P (Theorem 3.1) by dense eigendecomposition or ARPACK (the paper's own
    choice for lambda, Section 6.1).
"""

from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "geer_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
# The mutation tests point this at a copy of the checker built with a planted
# mistake, to show that the pins catch it.
_LIB_OVERRIDE = os.environ.get("GEER_ORACLE_LIB")
_lib = None

_i32p = np.ctypeslib.ndpointer(dtype=np.int32, flags="C_CONTIGUOUS")
_i64p = np.ctypeslib.ndpointer(dtype=np.int64, flags="C_CONTIGUOUS")
_f64p = np.ctypeslib.ndpointer(dtype=np.float64, flags="C_CONTIGUOUS")
_u32p = np.ctypeslib.ndpointer(dtype=np.uint32, flags="C_CONTIGUOUS")
_u8p = np.ctypeslib.ndpointer(dtype=np.uint8, flags="C_CONTIGUOUS")

STATS_DTYPE = np.dtype([
    ("ell", np.int32), ("ell_b", np.int32), ("lf", np.int32), ("batches_run", np.int32),
    ("eta1", np.int64), ("walk_pairs", np.int64), ("supp_sum", np.int64),
    ("r_b", np.float64), ("r_f", np.float64), ("r", np.float64), ("psi", np.float64),
    ("eta_star", np.float64), ("z_sum", np.float64), ("z2_sum", np.float64),
    ("var", np.float64), ("f_last", np.float64),
])


def build(force: bool = True) -> str:
    """Compile ``liboracle.so`` with the host C compiler (IEEE FP64, no fast-math)."""
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c11", "-fPIC", "-shared", "-o", tmp, _SRC,
                               "-lm", "-lpthread"])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def lib():
    global _lib
    if _lib is None:
        if _LIB_OVERRIDE:
            L = ctypes.CDLL(_LIB_OVERRIDE)
        else:
            if not os.path.exists(_LIB_PATH):
                build(force=True)
            L = ctypes.CDLL(_LIB_PATH)
        L.oracle_philox4x32_10.argtypes = [_u32p, _u32p, _u32p]
        L.oracle_smm_hop.argtypes = [ctypes.c_int64, _i64p, _i32p, _f64p, _f64p]
        L.oracle_top2.argtypes = [ctypes.c_int64, _f64p, ctypes.POINTER(ctypes.c_double),
                                  ctypes.POINTER(ctypes.c_double)]
        L.oracle_ell.argtypes = [ctypes.c_double] * 4
        L.oracle_ell.restype = ctypes.c_int32
        L.oracle_ell_peng.argtypes = [ctypes.c_double, ctypes.c_double]
        L.oracle_ell_peng.restype = ctypes.c_int32
        L.oracle_psi.argtypes = [ctypes.c_int32] + [ctypes.c_double] * 6
        L.oracle_psi.restype = ctypes.c_double
        L.oracle_eta_star.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_int32,
                                      ctypes.c_double]
        L.oracle_eta_star.restype = ctypes.c_double
        L.oracle_eta1.argtypes = [ctypes.c_double, ctypes.c_int32]
        L.oracle_eta1.restype = ctypes.c_uint64
        L.oracle_h.argtypes = [ctypes.c_double, ctypes.c_int32]
        L.oracle_h.restype = ctypes.c_double
        L.oracle_bernstein.argtypes = [ctypes.c_double] * 4
        L.oracle_bernstein.restype = ctypes.c_double
        L.oracle_walk_trace.argtypes = [_i64p, _i32p, ctypes.c_int32, ctypes.c_int32,
                                        ctypes.c_uint64, ctypes.c_uint32, ctypes.c_uint32,
                                        ctypes.c_uint32, ctypes.c_uint32, _i32p]
        L.oracle_amc.argtypes = [_i64p, _i32p, ctypes.c_int32, ctypes.c_int32, _f64p, _f64p,
                                 ctypes.c_int64, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                 ctypes.c_double, ctypes.c_uint64, ctypes.c_uint32,
                                 ctypes.c_void_p]
        L.oracle_amc.restype = ctypes.c_double
        L.oracle_geer.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i32p,
                                  _f64p, ctypes.c_double, ctypes.c_int32, ctypes.c_double,
                                  ctypes.c_uint64, ctypes.c_int32, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int32, _f64p, ctypes.c_void_p,
                                  ctypes.c_void_p, ctypes.c_int32]
        L.oracle_geer.restype = ctypes.c_int
        L.oracle_series.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p, _i32p,
                                    _i32p, ctypes.c_int32, _f64p]
        L.oracle_series.restype = ctypes.c_int
        L.oracle_exact_cg.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int64, _i32p,
                                      _i32p, ctypes.c_double, ctypes.c_int32, ctypes.c_int32,
                                      _f64p, _i32p]
        L.oracle_exact_cg.restype = ctypes.c_int
        L.oracle_smm_vectors.argtypes = [ctypes.c_int64, _i64p, _i32p, ctypes.c_int32,
                                         ctypes.c_int32, ctypes.c_int32, _f64p, _f64p, _u8p,
                                         ctypes.POINTER(ctypes.c_double)]
        L.oracle_amc_samples.argtypes = [_i64p, _i32p, ctypes.c_int32, ctypes.c_int32, _f64p,
                                         _f64p, ctypes.c_int32, ctypes.c_uint64,
                                         ctypes.c_uint32, ctypes.c_uint32, ctypes.c_int64, _f64p]
        L.oracle_stats_size.restype = ctypes.c_int
        if L.oracle_stats_size() != STATS_DTYPE.itemsize:
            raise RuntimeError("oracle stats layout mismatch")
        _lib = L
    return _lib


def _csr(row_ptr, col_idx):
    return (np.ascontiguousarray(row_ptr, dtype=np.int64),
            np.ascontiguousarray(col_idx, dtype=np.int32))


def _default_threads() -> int:
    return max(1, min(16, os.cpu_count() or 1))


# ---------------------------------------------------------------------------
# Philox and walks
# ---------------------------------------------------------------------------

def philox4x32_10(counter, key) -> np.ndarray:
    """Philox4x32-10 block: 4 x uint32 counter, 2 x uint32 key -> 4 x uint32."""
    c = np.ascontiguousarray(counter, dtype=np.uint32).reshape(4)
    k = np.ascontiguousarray(key, dtype=np.uint32).reshape(2)
    out = np.zeros(4, dtype=np.uint32)
    lib().oracle_philox4x32_10(c, k, out)
    return out


def walk_trace(row_ptr, col_idx, start: int, lf: int, seed: int, q: int, batch: int, k: int,
               side: int) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    out = np.zeros(max(lf, 1), dtype=np.int32)
    lib().oracle_walk_trace(rp, ci, int(start), int(lf), int(seed), int(q), int(batch), int(k),
                            int(side), out)
    return out[:lf]


# ---------------------------------------------------------------------------
# Scalar formulas
# ---------------------------------------------------------------------------

def ell(ds: float, dt: float, eps: float, lam: float) -> int:
    return int(lib().oracle_ell(float(ds), float(dt), float(eps), float(lam)))


def ell_peng(eps: float, lam: float) -> int:
    return int(lib().oracle_ell_peng(float(eps), float(lam)))


def psi(lf, m1s, m2s, m1t, m2t, ds, dt) -> float:
    return float(lib().oracle_psi(int(lf), m1s, m2s, m1t, m2t, float(ds), float(dt)))


def eta_star(psi_v, eps, tau, delta) -> float:
    return float(lib().oracle_eta_star(float(psi_v), float(eps), int(tau), float(delta)))


def eta1(eta_star_v, tau) -> int:
    return int(lib().oracle_eta1(float(eta_star_v), int(tau)))


def h_budget(eta_star_v, tau) -> float:
    return float(lib().oracle_h(float(eta_star_v), int(tau)))


def bernstein(nz, var, psi_v, delta) -> float:
    return float(lib().oracle_bernstein(float(nz), float(var), float(psi_v), float(delta)))


def top2(x) -> tuple[float, float]:
    x = np.ascontiguousarray(x, dtype=np.float64)
    a = ctypes.c_double()
    b = ctypes.c_double()
    lib().oracle_top2(x.size, x, ctypes.byref(a), ctypes.byref(b))
    return a.value, b.value


# ---------------------------------------------------------------------------
# SMM, AMC, GEER
# ---------------------------------------------------------------------------

def smm_hop(row_ptr, col_idx, x) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.zeros_like(x)
    lib().oracle_smm_hop(rp.size - 1, rp, ci, x, y)
    return y


def smm_vectors(row_ptr, col_idx, s: int, t: int, hops: int):
    """(x, y, supp_x, supp_y, r_b) after ``hops`` products (Algorithm SMM)."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    x = np.zeros(n)
    y = np.zeros(n)
    supp = np.zeros(2 * n, dtype=np.uint8)
    rb = ctypes.c_double()
    lib().oracle_smm_vectors(n, rp, ci, int(s), int(t), int(hops), x, y, supp, ctypes.byref(rb))
    return x, y, supp[:n].astype(bool), supp[n:].astype(bool), rb.value


def amc(row_ptr, col_idx, s, t, x, y, eps, lf, tau=5, delta=0.01, seed=0, q=0):
    """Algorithm AMC with arbitrary non-negative input vectors -> (r_f, stats)."""
    rp, ci = _csr(row_ptr, col_idx)
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    st = np.zeros(1, dtype=STATS_DTYPE)
    rf = lib().oracle_amc(rp, ci, int(s), int(t), x, y, x.size, float(eps), int(lf), int(tau),
                          float(delta), int(seed), int(q), st.ctypes.data)
    return float(rf), st[0]


def amc_samples(row_ptr, col_idx, s, t, x, y, lf, seed, q, batch, count) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    out = np.zeros(count)
    lib().oracle_amc_samples(rp, ci, int(s), int(t), np.ascontiguousarray(x, dtype=np.float64),
                             np.ascontiguousarray(y, dtype=np.float64), int(lf), int(seed),
                             int(q), int(batch), int(count), out)
    return out


def geer(row_ptr, col_idx, s, t, eps, lam, *, tau=5, delta=0.01, seed=0, schedule="greedy",
         fixed_lb=None, qid=None, threads=None, tau_per_pair=None, ell_rule="paper"):
    """Algorithm GEER for arrays of pairs -> (r', stats record array).

    schedule: "greedy" (Eq. smm-amc) or "fixed" (exactly min(fixed_lb, l) SMM
    iterations per pair).  ``qid`` gives each pair's index in the walk
    counter (defaults to its position).  ell_rule: "paper" (Eq. ell, per
    pair) or "peng" (Eq. old-ell, the same l for every pair).
    """
    if ell_rule not in ("paper", "peng"):
        raise ValueError(ell_rule)
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    nq = s.size
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (nq,)))
    out = np.zeros(nq)
    st = np.zeros(nq, dtype=STATS_DTYPE)
    flb = None
    if schedule == "fixed":
        flb = np.ascontiguousarray(np.broadcast_to(np.asarray(fixed_lb, dtype=np.int32), (nq,)))
    elif schedule != "greedy":
        raise ValueError(schedule)
    q = None if qid is None else np.ascontiguousarray(qid, dtype=np.int64)
    tp = None
    if tau_per_pair is not None:
        tp = np.ascontiguousarray(np.broadcast_to(np.asarray(tau_per_pair, dtype=np.int32), (nq,)))
    rc = lib().oracle_geer(rp.size - 1, rp, ci, nq, s, t, e, float(lam), int(tau), float(delta),
                           int(seed), 0 if schedule == "greedy" else 1,
                           None if flb is None else flb.ctypes.data,
                           None if q is None else q.ctypes.data,
                           int(threads or _default_threads()), out, st.ctypes.data,
                           None if tp is None else tp.ctypes.data, 1 if ell_rule == "peng" else 0)
    if rc != 0:
        raise MemoryError("oracle_geer failed to allocate")
    return out, st


def series(row_ptr, col_idx, s, t, ell_v, threads=None) -> np.ndarray:
    """Truncated series r_l(s,t) of Eq. (r-ell) for per-pair l."""
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    ev = np.ascontiguousarray(np.broadcast_to(np.asarray(ell_v, dtype=np.int32), s.shape))
    out = np.zeros(s.size)
    lib().oracle_series(rp.size - 1, rp, ci, s.size, s, t, ev, int(threads or _default_threads()),
                        out)
    return out


def exact_cg(row_ptr, col_idx, s, t, tol=1e-12, max_iter=100000, threads=None):
    """Exact r(s,t) (Definition 2.1) by Jacobi-PCG -> (r, iterations)."""
    rp, ci = _csr(row_ptr, col_idx)
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    out = np.zeros(s.size)
    its = np.zeros(s.size, dtype=np.int32)
    rc = lib().oracle_exact_cg(rp.size - 1, rp, ci, s.size, s, t, float(tol), int(max_iter),
                               int(threads or _default_threads()), out, its)
    if rc != 0:
        raise MemoryError("oracle_exact_cg failed to allocate")
    return out, its


# ---------------------------------------------------------------------------
# Dense / library-routine parts (numpy LAPACK, scipy ARPACK)
# ---------------------------------------------------------------------------

def laplacian_dense(row_ptr, col_idx) -> np.ndarray:
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    A = np.zeros((n, n))
    for v in range(n):
        A[v, ci[rp[v]:rp[v + 1]]] = 1.0
    return np.diag(A.sum(axis=1)) - A


def exact_pinv(row_ptr, col_idx, s, t) -> np.ndarray:
    """Exact r(s,t) = (e_s - e_t) L^+ (e_s - e_t)^T (Definition 2.1), small graphs."""
    Lp = np.linalg.pinv(laplacian_dense(row_ptr, col_idx), hermitian=True)
    s = np.asarray(s)
    t = np.asarray(t)
    return Lp[s, s] + Lp[t, t] - Lp[s, t] - Lp[t, s]


def transition_eigs_dense(row_ptr, col_idx) -> np.ndarray:
    """All eigenvalues of P = D^-1 A, descending (via the similar D^-1/2 A D^-1/2)."""
    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    deg = np.diff(rp).astype(np.float64)
    A = np.zeros((n, n))
    for v in range(n):
        A[v, ci[rp[v]:rp[v + 1]]] = 1.0
    dm = 1.0 / np.sqrt(deg)
    N = dm[:, None] * A * dm[None, :]
    return np.sort(np.linalg.eigvalsh(N))[::-1]


def lambda_dense(row_ptr, col_idx) -> float:
    """lambda = max(|lambda_2|, |lambda_n|) of P (Theorem 3.1), dense eigensolver."""
    ev = transition_eigs_dense(row_ptr, col_idx)
    return float(max(abs(ev[1]), abs(ev[-1])))


def lambda_arpack(row_ptr, col_idx, tol=1e-10) -> float:
    """lambda of P by ARPACK (implicitly restarted Lanczos), as in Section 6.1."""
    import scipy.sparse as sp
    import scipy.sparse.linalg as sla

    rp, ci = _csr(row_ptr, col_idx)
    n = rp.size - 1
    deg = np.diff(rp).astype(np.float64)
    A = sp.csr_matrix((np.ones(ci.size), ci, rp), shape=(n, n))
    dm = sp.diags(1.0 / np.sqrt(deg))
    N = (dm @ A @ dm).tocsr()
    # deflate the known top eigenvector sqrt(d) (eigenvalue 1)
    u = np.sqrt(deg)
    u /= np.linalg.norm(u)

    def mv(v):
        v = np.asarray(v).ravel()
        w = N @ v
        return w - u * (u @ w)

    op = sla.LinearOperator((n, n), matvec=mv, dtype=np.float64)
    rng = np.random.default_rng(12345)
    v0 = rng.standard_normal(n)
    v0 -= u * (u @ v0)
    hi = sla.eigsh(op, k=1, which="LA", tol=tol, v0=v0, return_eigenvectors=False)[0]
    lo = sla.eigsh(op, k=1, which="SA", tol=tol, v0=v0, return_eigenvectors=False)[0]
    return float(max(abs(hi), abs(lo)))
