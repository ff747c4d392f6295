"""ctypes binding of ``libgeer.so`` -- argument marshalling only.

Every function here has the name of the C entry point it calls (see
``include/geer.h``); all computation happens in the HIP library.  There is no
CPU fallback: if the library is missing, importing this module raises.
"""

from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgeer.so")

GEER_OK = 0
GEER_E_INVALID_ARG = -1
GEER_E_GRAPH = -2
GEER_E_NOT_CONNECTED = -3
GEER_E_BIPARTITE = -4
GEER_E_NO_LAMBDA = -5
GEER_E_OOM = -6
GEER_E_DEVICE = -7
GEER_E_MODEL = -8

GEER_SCHEDULE_GREEDY = 0
GEER_SCHEDULE_LEARNED = 1
GEER_SCHEDULE_FIXED = 2

GEER_GRAPH_TRUSTED = 1
GEER_GRAPH_WIDE_WALK_RECORDS = 2

GEER_FLAG_FP64_VECTORS = 1
GEER_FLAG_GRAPH_LAUNCH = 2
GEER_FLAG_PENG_ELL = 4

GEER_STOP_SAME_NODE = 0
GEER_STOP_NO_WALKS = 1
GEER_STOP_BERNSTEIN = 2
GEER_STOP_CAP = 3

# Every symbol include/geer.h declares (checked by the CPU test-suite).
EXPORTED = [
    "geer_params_default", "geer_graph_create", "geer_graph_destroy", "geer_graph_set_lambda",
    "geer_graph_get_lambda", "geer_graph_compute_lambda", "geer_graph_info", "geer_query",
    "geer_query_device", "geer_smm", "geer_walk_traces", "geer_amc", "geer_last_error",
    "geer_version", "geer_model_create", "geer_model_free", "geer_model_save", "geer_model_load",
    "geer_model_get_params", "geer_model_set_params", "geer_model_set_norm",
    "geer_graph_set_costs", "geer_features", "geer_mlp_forward", "geer_mlp_grad",
    "geer_mlp_train", "geer_autotune", "geer_profile_enable", "geer_profile_read",
    "geer_amc_device_noalloc",
]

MLP_FEATURES = 14
MLP_HIDDEN = 64
MLP_OUTPUTS = 3
MLP_PARAMS = 14 * 64 + 64 + 64 * 64 + 64 + 64 * 3 + 3


class GeerError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"geer status {status}: {msg}")
        self.status = status


class geer_params(ctypes.Structure):
    _fields_ = [
        ("delta", ctypes.c_double),
        ("tau", ctypes.c_int32),
        ("schedule", ctypes.c_int32),
        ("seed", ctypes.c_uint64),
        ("qid_offset", ctypes.c_int64),
        ("fixed_ell_b", ctypes.c_void_p),
        ("model", ctypes.c_void_p),
        ("stream", ctypes.c_void_p),
        ("batch_queries", ctypes.c_int32),
        ("col_tile", ctypes.c_int32),
        ("walk_ilp", ctypes.c_int32),
        ("group_batches", ctypes.c_int32),
        ("flags", ctypes.c_uint32),
        ("reserved", ctypes.c_int32 * 7),
    ]


class geer_query_stats(ctypes.Structure):
    _fields_ = [
        ("ell", ctypes.c_int32), ("ell_b", ctypes.c_int32), ("tau", ctypes.c_int32),
        ("batches_run", ctypes.c_int32), ("stop_reason", ctypes.c_int32),
        ("fallback", ctypes.c_int32), ("eta1", ctypes.c_int64), ("walk_pairs", ctypes.c_int64),
        ("supp_sum", ctypes.c_int64), ("r_b", ctypes.c_double), ("r_f", ctypes.c_double),
        ("psi", ctypes.c_double), ("eta_star", ctypes.c_double), ("sigma2", ctypes.c_double),
        ("f_last", ctypes.c_double),
    ]


class geer_kernel_profile(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char * 32), ("launches", ctypes.c_int64),
                ("total_ms", ctypes.c_double), ("alg_bytes", ctypes.c_double),
                ("work_units", ctypes.c_double)]


STATS_DTYPE = np.dtype([(name, np.dtype(ctype)) for name, ctype in [
    ("ell", np.int32), ("ell_b", np.int32), ("tau", np.int32), ("batches_run", np.int32),
    ("stop_reason", np.int32), ("fallback", np.int32), ("eta1", np.int64),
    ("walk_pairs", np.int64), ("supp_sum", np.int64), ("r_b", np.float64), ("r_f", np.float64),
    ("psi", np.float64), ("eta_star", np.float64), ("sigma2", np.float64),
    ("f_last", np.float64)]])

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_u32 = ctypes.c_uint32
_u64 = ctypes.c_uint64
_f64 = ctypes.c_double

_SIGNATURES = {
    "geer_params_default": ([_vp], _i32),
    "geer_graph_create": ([_i32, _vp, _vp, _u32, ctypes.POINTER(_vp)], _i32),
    "geer_graph_destroy": ([_vp], None),
    "geer_graph_set_lambda": ([_vp, _f64], _i32),
    "geer_graph_get_lambda": ([_vp, ctypes.POINTER(_f64)], _i32),
    "geer_graph_compute_lambda": ([_vp, _i32, _f64, _u64, ctypes.POINTER(_f64)], _i32),
    "geer_graph_info": ([_vp, ctypes.POINTER(_i32), ctypes.POINTER(_i64), ctypes.POINTER(_i32)], _i32),
    "geer_query": ([_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "geer_query_device": ([_vp, _i64, _vp, _vp, _vp, _vp, _vp, _vp], _i32),
    "geer_smm": ([_vp, _i32, _vp, _vp, _i32, _u32, _i32, _vp, _vp, _vp, _vp], _i32),
    "geer_walk_traces": ([_vp, _i32, _vp, _vp, _vp, _vp, _vp, _i32, _u64, _vp], _i32),
    "geer_amc": ([_vp, _i32, _i32, _vp, _vp, _f64, _i32, _i32, _f64, _u64, _u32, _u32, _vp, _vp], _i32),
    "geer_amc_device_noalloc": ([_vp, _i32, _i32, _vp, _f64, _i32, _i32, _f64, _u64, _u32, _u32, _vp,
                                 _vp, _vp], _i32),
    "geer_last_error": ([], ctypes.c_char_p),
    "geer_version": ([], ctypes.c_char_p),
    "geer_model_create": ([_u64, ctypes.POINTER(_vp)], _i32),
    "geer_model_free": ([_vp], None),
    "geer_model_save": ([_vp, ctypes.c_char_p], _i32),
    "geer_model_load": ([ctypes.c_char_p, ctypes.POINTER(_vp)], _i32),
    "geer_model_get_params": ([_vp, _vp, _i64], _i32),
    "geer_model_set_params": ([_vp, _vp, _i64], _i32),
    "geer_model_set_norm": ([_vp, _vp, _vp, _vp, _vp], _i32),
    "geer_graph_set_costs": ([_vp, _f64, _f64], _i32),
    "geer_features": ([_vp, _i64, _vp, _vp, _vp, _vp], _i32),
    "geer_mlp_forward": ([_vp, _i64, _vp, _i32, _vp], _i32),
    "geer_mlp_grad": ([_vp, _i32, _vp, _vp, _vp, _vp], _i32),
    "geer_mlp_train": ([_vp, _i64, _vp, _vp, _vp, _i32, _i32, _f64, _vp, _vp], _i32),
    "geer_autotune": ([_vp, _i64, _vp, _vp, _vp, ctypes.c_char_p, _vp], _i32),
    "geer_profile_enable": ([_vp, _i32], _i32),
    "geer_profile_read": ([_vp, _vp, _i32, ctypes.POINTER(_i32)], _i32),
}


def _load():
    # torch ships its own HIP runtime with the same soname as the system one.
    # Loading torch first makes libgeer bind to that already-loaded runtime, so
    # one process never holds two HIP runtimes (device pointers and streams
    # from torch are then valid in the library).
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    if not os.path.exists(LIB_PATH):
        raise ImportError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2312_06123_amd.build`")
    lib = ctypes.CDLL(LIB_PATH)
    for name, (args, res) in _SIGNATURES.items():
        fn = getattr(lib, name, None)
        if fn is None:
            continue
        fn.argtypes = args
        fn.restype = res
    return lib


_lib = _load()


def lib():
    return _lib


def _check(status: int):
    if status != GEER_OK:
        raise GeerError(status, _lib.geer_last_error().decode(errors="replace"))


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.c_void_p)


def geer_version() -> str:
    return _lib.geer_version().decode()


def geer_last_error() -> str:
    return _lib.geer_last_error().decode(errors="replace")


def geer_params_default(**overrides) -> geer_params:
    p = geer_params()
    _check(_lib.geer_params_default(ctypes.byref(p)))
    for k, v in overrides.items():
        setattr(p, k, v)
    return p


def geer_graph_create(n: int, row_ptr, col_idx, flags: int = 0) -> ctypes.c_void_p:
    rp = np.ascontiguousarray(row_ptr, dtype=np.int32)
    ci = np.ascontiguousarray(col_idx, dtype=np.int32)
    out = ctypes.c_void_p()
    _check(_lib.geer_graph_create(int(n), _ptr(rp), _ptr(ci), int(flags), ctypes.byref(out)))
    return out


def geer_graph_destroy(g) -> None:
    _lib.geer_graph_destroy(g)


def geer_graph_set_lambda(g, lam: float) -> None:
    _check(_lib.geer_graph_set_lambda(g, float(lam)))


def geer_graph_get_lambda(g) -> float:
    v = ctypes.c_double()
    _check(_lib.geer_graph_get_lambda(g, ctypes.byref(v)))
    return v.value


def geer_graph_compute_lambda(g, max_iter: int = 300, tol: float = 1e-9, seed: int = 1) -> float:
    v = ctypes.c_double()
    _check(_lib.geer_graph_compute_lambda(g, int(max_iter), float(tol), int(seed), ctypes.byref(v)))
    return v.value


def geer_graph_info(g):
    n, nnz, md = ctypes.c_int32(), ctypes.c_int64(), ctypes.c_int32()
    _check(_lib.geer_graph_info(g, ctypes.byref(n), ctypes.byref(nnz), ctypes.byref(md)))
    return n.value, nnz.value, md.value


def geer_query(g, s, t, eps, params: geer_params | None = None, stats: bool = False,
               fixed_ell_b=None):
    """Host-array query.  Returns r (float64[nq]) or (r, stats record array)."""
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    nq = s.size
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), (nq,)))
    p = params if params is not None else geer_params_default()
    keep = None
    if fixed_ell_b is not None:
        # a copy: the caller's params must not keep a pointer to `keep`
        p = geer_params.from_buffer_copy(p)
        keep = np.ascontiguousarray(np.broadcast_to(np.asarray(fixed_ell_b, dtype=np.int32), (nq,)))
        p.fixed_ell_b = keep.ctypes.data
        p.schedule = GEER_SCHEDULE_FIXED
    r = np.zeros(nq)
    st = np.zeros(nq, dtype=STATS_DTYPE) if stats else None
    _check(_lib.geer_query(g, nq, _ptr(s), _ptr(t), _ptr(e), ctypes.byref(p), _ptr(r),
                           _ptr(st) if st is not None else None))
    del keep
    return (r, st) if stats else r


def geer_query_device(g, s, t, eps, r_out, params: geer_params | None = None, stats_out=None):
    """Device-array query on torch tensors (int32 s/t, float64 eps/r_out on the GPU).
    ``stats_out``: optional uint8 tensor of nq * sizeof(geer_query_stats) bytes."""
    import torch

    nq = s.numel()
    for name, x, dt in (("s", s, torch.int32), ("t", t, torch.int32), ("eps", eps, torch.float64),
                        ("r_out", r_out, torch.float64)):
        if x.dtype != dt or not x.is_cuda or not x.is_contiguous() or x.numel() != nq:
            raise ValueError(f"{name} must be a contiguous {dt} GPU tensor of {nq} elements")
    p = params if params is not None else geer_params_default()
    if not p.stream:
        # a copy: the caller's params keep "no stream" (torch's current one at each call)
        p = geer_params.from_buffer_copy(p)
        p.stream = torch.cuda.current_stream().cuda_stream
    sp = None
    if stats_out is not None:
        if stats_out.numel() < nq * ctypes.sizeof(geer_query_stats) or not stats_out.is_cuda:
            raise ValueError("stats_out too small")
        sp = ctypes.c_void_p(stats_out.data_ptr())
    _check(_lib.geer_query_device(g, nq, ctypes.c_void_p(s.data_ptr()), ctypes.c_void_p(t.data_ptr()),
                                  ctypes.c_void_p(eps.data_ptr()), ctypes.byref(p),
                                  ctypes.c_void_p(r_out.data_ptr()), sp))


def geer_smm(g, s, t, hops: int, fp64: bool = False, col_tile: int = 0):
    """Returns (vectors [n, 2nq], r_b [nq], top2 [nq, 4], supp [nq, 2])."""
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    nq = s.size
    n, _, _ = geer_graph_info(g)
    vec = np.zeros((n, 2 * nq), dtype=np.float64 if fp64 else np.float32)
    rb = np.zeros(nq)
    top2 = np.zeros((nq, 4))
    supp = np.zeros((nq, 2), dtype=np.int64)
    _check(_lib.geer_smm(g, nq, _ptr(s), _ptr(t), int(hops),
                         GEER_FLAG_FP64_VECTORS if fp64 else 0, int(col_tile), _ptr(vec), _ptr(rb),
                         _ptr(top2), _ptr(supp)))
    return vec, rb, top2, supp


def geer_walk_traces(g, start, q, batch, k, side, lf: int, seed: int) -> np.ndarray:
    start = np.ascontiguousarray(start, dtype=np.int32)
    nw = start.size
    arr = [np.ascontiguousarray(np.broadcast_to(np.asarray(a, dtype=np.uint32), (nw,)))
           for a in (q, batch, k, side)]
    out = np.zeros((nw, max(lf, 1)), dtype=np.int32)
    _check(_lib.geer_walk_traces(g, nw, _ptr(start), *[_ptr(a) for a in arr], int(lf), int(seed),
                                 _ptr(out)))
    return out[:, :lf]


def geer_amc(g, s: int, t: int, x, y, eps: float, lf: int, tau: int = 5, delta: float = 0.01,
             seed: int = 0, q: int = 0, fp64: bool = False):
    x = np.ascontiguousarray(x, dtype=np.float64)
    y = np.ascontiguousarray(y, dtype=np.float64)
    rf = ctypes.c_double()
    st = np.zeros(1, dtype=STATS_DTYPE)
    _check(_lib.geer_amc(g, int(s), int(t), _ptr(x), _ptr(y), float(eps), int(lf), int(tau),
                         float(delta), int(seed), int(q), GEER_FLAG_FP64_VECTORS if fp64 else 0,
                         ctypes.byref(rf), _ptr(st)))
    return rf.value, st[0]


def geer_amc_device_noalloc(g, s: int, t: int, d_xy: int, eps: float, lf: int, d_rf: int,
                            d_stats: int = 0, tau: int = 5, delta: float = 0.01, seed: int = 0,
                            q: int = 0, fp64: bool = False, stream: int = 0) -> None:
    """geer_amc on device memory with no allocation: d_xy (2n interleaved
    values), d_rf (one double) and d_stats (one record, or 0) are device
    addresses; stream is a hipStream_t handle or 0 for the library stream."""
    _check(_lib.geer_amc_device_noalloc(g, int(s), int(t), ctypes.c_void_p(d_xy), float(eps), int(lf),
                                        int(tau), float(delta), int(seed), int(q),
                                        GEER_FLAG_FP64_VECTORS if fp64 else 0,
                                        ctypes.c_void_p(stream or None), ctypes.c_void_p(d_rf),
                                        ctypes.c_void_p(d_stats or None)))


def geer_profile_enable(g, on: bool = True) -> None:
    _check(_lib.geer_profile_enable(g, 1 if on else 0))


def geer_profile_read(g) -> dict:
    """{kernel name: {launches, total_ms, alg_bytes, work_units}}."""
    recs = (geer_kernel_profile * 32)()
    cnt = ctypes.c_int32()
    _check(_lib.geer_profile_read(g, recs, 32, ctypes.byref(cnt)))
    return {r.name.decode(): {"launches": r.launches, "total_ms": r.total_ms,
                              "alg_bytes": r.alg_bytes, "work_units": r.work_units}
            for r in recs[:cnt.value]}


class geer_tuning(ctypes.Structure):
    _fields_ = [("col_tile", ctypes.c_int32), ("from_cache", ctypes.c_int32),
                ("ns_per_walk_step", ctypes.c_double), ("ns_per_hop2_unit", ctypes.c_double),
                ("ns_per_dense_hop", ctypes.c_double), ("rho2", ctypes.c_double),
                ("rhod", ctypes.c_double)]


def geer_autotune(g, s, t, eps, cache_path: str | None = None) -> dict:
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), s.shape))
    out = geer_tuning()
    _check(_lib.geer_autotune(g, s.size, _ptr(s), _ptr(t), _ptr(e),
                              cache_path.encode() if cache_path else None, ctypes.byref(out)))
    return {k: getattr(out, k) for k, _ in geer_tuning._fields_}


def geer_graph_set_costs(g, rho2: float, rhod: float) -> None:
    _check(_lib.geer_graph_set_costs(g, float(rho2), float(rhod)))


def geer_features(g, s, t, eps) -> np.ndarray:
    s = np.ascontiguousarray(s, dtype=np.int32)
    t = np.ascontiguousarray(t, dtype=np.int32)
    e = np.ascontiguousarray(np.broadcast_to(np.asarray(eps, dtype=np.float64), s.shape))
    out = np.zeros((s.size, MLP_FEATURES), dtype=np.float32)
    _check(_lib.geer_features(g, s.size, _ptr(s), _ptr(t), _ptr(e), _ptr(out)))
    return out


class Model:
    """Owning wrapper of a geer_model handle (the learned scheduler)."""

    def __init__(self, seed: int = 0, path: str | None = None):
        self.handle = ctypes.c_void_p()
        if path is not None:
            _check(_lib.geer_model_load(path.encode(), ctypes.byref(self.handle)))
        else:
            _check(_lib.geer_model_create(int(seed), ctypes.byref(self.handle)))

    def close(self):
        if self.handle:
            _lib.geer_model_free(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def save(self, path: str) -> None:
        _check(_lib.geer_model_save(self.handle, path.encode()))

    def get_params(self) -> np.ndarray:
        out = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_lib.geer_model_get_params(self.handle, _ptr(out), MLP_PARAMS))
        return out

    def set_params(self, p) -> None:
        p = np.ascontiguousarray(p, dtype=np.float32)
        _check(_lib.geer_model_set_params(self.handle, _ptr(p), p.size))

    def set_norm(self, mean, std, lo, hi) -> None:
        arr = [np.ascontiguousarray(a, dtype=np.float32) for a in (mean, std, lo, hi)]
        _check(_lib.geer_model_set_norm(self.handle, *[_ptr(a) for a in arr]))

    def forward(self, x, bf16: bool = False) -> np.ndarray:
        x = np.ascontiguousarray(x, dtype=np.float32)
        y = np.zeros((x.shape[0], MLP_OUTPUTS), dtype=np.float32)
        _check(_lib.geer_mlp_forward(self.handle, x.shape[0], _ptr(x), 1 if bf16 else 0, _ptr(y)))
        return y

    def grad(self, x, y, w) -> np.ndarray:
        x, y, w = [np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, w)]
        g = np.zeros(MLP_PARAMS, dtype=np.float32)
        _check(_lib.geer_mlp_grad(self.handle, x.shape[0], _ptr(x), _ptr(y), _ptr(w), _ptr(g)))
        return g

    def train(self, x, y, w, steps: int, batch: int = 64, lr: float = 1e-3, order=None):
        x, y, w = [np.ascontiguousarray(a, dtype=np.float32) for a in (x, y, w)]
        loss = np.zeros(max(steps, 1), dtype=np.float32)
        o = None if order is None else np.ascontiguousarray(order, dtype=np.int64)
        _check(_lib.geer_mlp_train(self.handle, x.shape[0], _ptr(x), _ptr(y), _ptr(w), int(steps),
                                   int(batch), float(lr), _ptr(o) if o is not None else None,
                                   _ptr(loss)))
        return loss[:steps]


class Graph:
    """Owning wrapper of a geer_graph handle."""

    def __init__(self, n, row_ptr, col_idx, flags: int = 0, lam: float | None = None):
        self.handle = geer_graph_create(n, row_ptr, col_idx, flags)
        self.n = int(n)
        if lam is not None:
            geer_graph_set_lambda(self.handle, lam)

    def close(self):
        if self.handle:
            geer_graph_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()
