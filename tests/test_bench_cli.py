"""bench.py on the CPU: more than one GPU is refused with a message and a
non-zero status before any device work; the roofline entry takes the
dominant kernel's algorithmic rate, and measured traffic is reported only
while the kernel source matches the one the counters were taken on."""

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
    monkeypatch.setattr(b, "measured_traffic", lambda kernel: 2e9 if kernel == "walk" else None)
    prof = {
        "walk": {"launches": 20, "total_ms": 10.0, "alg_bytes": 4e9, "work_units": 1e8},
        "hop_light": {"launches": 2, "total_ms": 1.0, "alg_bytes": 1e9, "work_units": 0},
        "epilogue": {"launches": 5, "total_ms": 30.0, "alg_bytes": 0.0, "work_units": 0},  # no bytes
        "unused": {"launches": 0, "total_ms": 0.0, "alg_bytes": 0.0, "work_units": 0},
    }
    roof, table = b.roofline_of(prof, steps=2)
    assert roof["kernel"] == "walk"  # the longest kernel that moves counted bytes
    assert roof["achieved"] == round(4e9 / 10e-3 / 1e9, 2)
    assert roof["frac"] == round(roof["achieved"] / b.HBM_PEAK_GBS, 4)
    assert roof["alg_bytes_per_launch"] == 4e9 / 20
    assert roof["avg_launch_us"] == 500.0
    assert roof["traffic"] == 2e9
    assert roof["traffic_GBs"] == round(2e9 / 500e-6 / 1e9, 1)  # bytes moved per launch / launch time
    assert roof["traffic_frac"] == round(roof["traffic_GBs"] / b.HBM_PEAK_GBS, 4)
    assert "unused" not in table and table["walk"]["launches_per_step"] == 10
    assert table["walk"]["units_per_launch"] == 1e8 / 20


def test_measured_traffic_follows_the_source_hash(tmp_path, monkeypatch):
    import hashlib
    import json

    b = _bench_module()
    src = tmp_path / "k.hip"
    src.write_text("kernel source")
    (tmp_path / "profiles").mkdir()
    rec = {"walk": {"source": "k.hip", "traffic_bytes_per_launch": 123.0,
                    "source_sha256_16": hashlib.sha256(b"kernel source").hexdigest()[:16]}}
    (tmp_path / "profiles" / "traffic.json").write_text(json.dumps(rec))
    monkeypatch.setattr(b, "ROOT", str(tmp_path))
    assert b.measured_traffic("walk") == 123.0
    src.write_text("kernel source, changed")  # counters taken on other code: no traffic
    assert b.measured_traffic("walk") is None
    assert b.measured_traffic("missing") is None
