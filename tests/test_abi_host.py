"""CPU-side checks of the host parts of the C ABI: parameter defaults, the
argument checks every entry point makes before any device work, and the
learned-scheduler model object (kept in host memory until first used on a
device): creation, parameters, normalisation and checkpoints."""

import ctypes
import os

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
G = pytest.importorskip("paper_2312_06123_amd.geer")


def _status(call):
    with pytest.raises(G.GeerError) as e:
        call()
    return e.value.status


def test_params_defaults():
    p = G.geer_params_default()
    assert p.delta == 0.01 and p.tau == 5  # Section 6.1 defaults
    assert p.schedule == G.GEER_SCHEDULE_GREEDY and p.seed == 0 and p.flags == 0
    assert p.batch_queries == 0 and p.col_tile == 0 and p.group_batches == 0 and p.walk_ilp == 0


def test_null_graph_rejected_by_every_entry_point():
    lib = G.lib()
    null = None
    s = np.zeros(1, np.int32)
    e = np.ones(1)
    r = np.zeros(1)
    vp = ctypes.c_void_p
    checks = [
        lib.geer_query(null, 1, s.ctypes.data, s.ctypes.data, e.ctypes.data, None, r.ctypes.data, None),
        lib.geer_query_device(null, 1, s.ctypes.data, s.ctypes.data, e.ctypes.data, None, r.ctypes.data,
                              None),
        lib.geer_smm(null, 1, s.ctypes.data, s.ctypes.data, 1, 0, 0, r.ctypes.data, None, None, None),
        lib.geer_amc(null, 0, 1, r.ctypes.data, r.ctypes.data, 0.1, 3, 5, 0.01, 0, 0, 0, r.ctypes.data,
                     None),
        lib.geer_walk_traces(null, 1, s.ctypes.data, s.ctypes.data, s.ctypes.data, s.ctypes.data,
                             s.ctypes.data, 3, 0, s.ctypes.data),
        lib.geer_graph_set_lambda(null, 0.5),
        lib.geer_graph_compute_lambda(null, 10, 1e-6, 1, ctypes.byref(ctypes.c_double())),
        lib.geer_features(null, 1, s.ctypes.data, s.ctypes.data, e.ctypes.data, r.ctypes.data),
        lib.geer_graph_set_costs(null, 1.0, 1.0),
        lib.geer_autotune(null, 1, s.ctypes.data, s.ctypes.data, e.ctypes.data, None, None),
        lib.geer_profile_enable(null, 1),
    ]
    assert all(c == G.GEER_E_INVALID_ARG for c in checks), checks
    assert lib.geer_graph_get_lambda(null, ctypes.byref(ctypes.c_double())) == G.GEER_E_INVALID_ARG
    lib.geer_graph_destroy(null)  # ignored
    assert G.geer_last_error() != ""


def test_model_parameters_and_checkpoint_roundtrip(tmp_path):
    m = G.Model(seed=42)
    p = m.get_params()
    assert p.shape == (G.MLP_PARAMS,) and np.all(np.isfinite(p))
    # He-uniform: weights bounded by sqrt(6 / fan_in), biases zero
    F, H, O = G.MLP_FEATURES, G.MLP_HIDDEN, G.MLP_OUTPUTS
    w1, b1 = p[:F * H], p[F * H:F * H + H]
    assert np.all(np.abs(w1) <= np.sqrt(6.0 / F)) and np.all(b1 == 0)
    assert G.Model(seed=42).get_params().tobytes() == p.tobytes()  # seeded
    assert G.Model(seed=43).get_params().tobytes() != p.tobytes()
    q = (p * 0.5).astype(np.float32)
    m.set_params(q)
    assert np.array_equal(m.get_params(), q)
    mean = np.arange(F, dtype=np.float32)
    std = np.full(F, 2.0, np.float32)
    m.set_norm(mean, std, mean - 1, mean + 1)
    path = str(tmp_path / "m.geermlp")
    m.save(path)
    m2 = G.Model(path=path)
    assert np.array_equal(m2.get_params(), q)
    # wrong counts, bad normalisation and unreadable checkpoints are rejected
    assert _status(lambda: m.set_params(q[:-1])) == G.GEER_E_INVALID_ARG
    assert _status(lambda: m.set_norm(mean, np.zeros(F), mean, mean)) == G.GEER_E_INVALID_ARG
    bad = tmp_path / "bad.geermlp"
    bad.write_bytes(open(path, "rb").read()[:100])
    assert _status(lambda: G.Model(path=str(bad))) == G.GEER_E_MODEL
    assert _status(lambda: G.Model(path=str(tmp_path / "missing.geermlp"))) == G.GEER_E_MODEL


def test_shipped_scheduler_checkpoint_loads():
    m = G.Model(path=os.path.join(ROOT, "paper_2312_06123_amd", "data", "scheduler.geermlp"))
    p = m.get_params()
    assert np.all(np.isfinite(p)) and np.abs(p).max() > 0


def test_fixed_depths_do_not_leak_into_caller_params():
    # geer_query(..., fixed_ell_b=...) works on a copy of the parameters: the
    # caller's object keeps its schedule and holds no pointer to the depths
    p = G.geer_params_default(seed=5)
    q = G.geer_params.from_buffer_copy(p)
    with pytest.raises(G.GeerError):  # no graph: the call fails its argument check
        G.geer_query(None, np.array([0], np.int32), np.array([1], np.int32), 0.1, p,
                     fixed_ell_b=np.array([2], np.int32))
    assert bytes(p) == bytes(q)
    assert p.schedule == G.GEER_SCHEDULE_GREEDY and not p.fixed_ell_b
