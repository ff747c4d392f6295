"""bench.py on the CPU: more than one GPU is refused with a message and a
non-zero status before any device work; the roofline entry takes the
dominant kernel's algorithmic rate (walk steps at 20 bytes), and measured
traffic is reported only for the workload and sources the counters were
taken on."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_bench_refuses_more_than_one_gpu():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert p.returncode == 2
    assert "one GPU" in p.stderr
    assert p.stdout.strip() == ""


def _bench_module():
    import importlib.util

    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_roofline_takes_the_dominant_kernel_and_its_algorithmic_rate(monkeypatch):
    b = _bench_module()
    monkeypatch.setattr(b, "measured_traffic", lambda kernel, wl: 2e9 if kernel == "walk" else None)
    prof = {
        "walk": {"launches": 20, "total_ms": 10.0, "alg_bytes": 4e9, "work_units": 1e8},
        "hop_light": {"launches": 2, "total_ms": 1.0, "alg_bytes": 1e9, "work_units": 0},
        "epilogue": {"launches": 5, "total_ms": 30.0, "alg_bytes": 0.0, "work_units": 0},  # no bytes
        "unused": {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0, "work_units": 0},
    }
    roof, table = b.roofline_of(prof, steps=2, workload={})
    assert roof["kernel"] == "walk"  # the longest kernel that moves counted bytes
    # walk steps are priced at 20 bytes each (offsets 8, index 4, two FP32 values 8)
    per_launch = 20.0 * 1e8 / 20
    assert roof["alg_bytes_per_launch"] == per_launch
    assert roof["achieved"] == round(per_launch / 500e-6 / 1e9, 2)
    assert roof["frac"] == round(roof["achieved"] / b.HBM_PEAK_GBS, 4)
    assert roof["packed_record_model"]["alg_bytes_per_launch"] == 4e9 / 20
    assert roof["avg_launch_us"] == 500.0
    assert roof["traffic"] == 2e9
    assert roof["traffic_GBs"] == round(2e9 / 500e-6 / 1e9, 1)  # bytes moved per launch / launch time
    assert roof["traffic_frac"] == round(roof["traffic_GBs"] / b.HBM_PEAK_GBS, 4)
    assert "unused" not in table and table["walk"]["launches_per_step"] == 10
    assert table["walk"]["units_per_launch"] == 1e8 / 20
    # an SpMM-dominated profile takes the library's byte count
    prof["walk"]["total_ms"] = 0.5
    roof, _ = b.roofline_of(prof, steps=2, workload={})
    assert roof["kernel"] == "hop_light" and roof["alg_bytes_per_launch"] == 1e9 / 2


def test_measured_traffic_follows_workload_and_sources(tmp_path, monkeypatch):
    import json

    b = _bench_module()
    wl = {"graph": "chung-lu n=1000000 seed=1002", "pairs": "uniform", "schedule": "learned"}
    rec = {"walk": {"traffic_bytes_per_launch": 123.0, "workload": wl, "sources": b.source_hashes()}}
    (tmp_path / "profiles").mkdir()
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    real_root = b.ROOT
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    monkeypatch.setattr(b, "source_hashes", lambda: rec["walk"]["sources"])
    assert b.measured_traffic("walk", wl) == 123.0
    # another workload (edge pairs, another schedule, tile or graph): no traffic
    assert b.measured_traffic("walk", dict(wl, pairs="edge")) is None
    assert b.measured_traffic("walk", dict(wl, schedule="plain")) is None
    assert b.measured_traffic("missing", wl) is None
    # counters taken on other code: no traffic
    changed = dict(rec["walk"]["sources"])
    changed[next(iter(changed))] = "0" * 16
    monkeypatch.setattr(b, "source_hashes", lambda: changed)
    assert b.measured_traffic("walk", wl) is None
    monkeypatch.setattr(b, "ROOT", real_root)


def test_cpu_threads_respect_the_allotted_share(monkeypatch):
    b = _bench_module()
    monkeypatch.setenv("OMP_NUM_THREADS", "3")
    assert b.host_threads() == min(3, len(os.sched_getaffinity(0)))
    monkeypatch.delenv("OMP_NUM_THREADS")
    assert b.host_threads() == len(os.sched_getaffinity(0))
    assert isinstance(b.cpu_model(), str) and b.cpu_model()
