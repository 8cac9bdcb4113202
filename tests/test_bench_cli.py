"""bench.py's command-line contract on the CPU: a request for more than one GPU
exits with a message (this build runs on one GPU), and the measured-traffic lookup
applies only to the kernel code, per-event energy, precision and run settings it
was measured with (on any sample size of the batch)."""
import importlib.util
import json
import os
import subprocess
import sys
import types

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode != 0
    msg = json.loads(r.stdout.strip().splitlines()[-1])
    assert "one GPU" in msg["error"]


def _bench():
    spec = importlib.util.spec_from_file_location("bench_mod", os.path.join(ROOT, "bench.py"))
    m = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(m)
    return m


def test_traffic_applies_only_to_its_settings(tmp_path, monkeypatch):
    b = _bench()
    src = tmp_path / "k.hip"
    src.write_text("int k() { return 1; }\n")
    t = {"kernel_source": str(src), "kernel_code_sha256": b.kernel_source_digest(str(src)),
         "precision": "fp64", "events": 1000, "energy_MeV": 10000.0, "energy_budget_MeV": 1e8,
         "pool_slots": 1 << 24, "iterations_per_sync": 4, "bytes_per_iteration": 123.0}
    (tmp_path / "w_traffic.json").write_text(json.dumps(t))
    monkeypatch.setattr(b, "TRAFFIC_GLOB", str(tmp_path / "*_traffic.json"))
    base = dict(precision="fp64", events=1000, energy=10000.0, budget=1e8, pool=1 << 24, per_sync=4)
    assert b.measured_traffic(types.SimpleNamespace(**base)) == 123.0
    for k, v in (("precision", "mixed"), ("energy", 1.0), ("budget", 1.0),
                 ("per_sync", 1), ("pool", 64)):
        assert b.measured_traffic(types.SimpleNamespace(**{**base, k: v})) is None
    # a sample of the batch with the same per-event settings: the counters carry over
    assert b.measured_traffic(types.SimpleNamespace(**{**base, "events": 10})) == 123.0
    src.write_text("int k() { return 2; }\n")  # the kernel code changed since
    assert b.measured_traffic(types.SimpleNamespace(**base)) is None


def test_layer_comparison_bar():
    b = _bench()
    rng = np.random.default_rng(0)
    o = rng.normal(10.0, 1.0, (400, 100))
    g = o + rng.normal(0, 1e-3, o.shape)
    worst, ok = b.compare_layers(g, o, 1e-3)
    assert ok and worst < 1
    worst, ok = b.compare_layers(g * 1.05, o, 1e-3)  # 5 % too high everywhere
    assert not ok and worst > 1


def test_kernel_digest_ignores_comments(tmp_path):
    b = _bench()
    a = tmp_path / "a.hip"
    c = tmp_path / "b.hip"
    a.write_text("int f() { return 1; }  // one\n/* block */\n")
    c.write_text("int f()   {\n  return 1;\n}\n")
    assert b.kernel_source_digest(str(a)) == b.kernel_source_digest(str(c))
    c.write_text("int f() { return 2; }\n")
    assert b.kernel_source_digest(str(a)) != b.kernel_source_digest(str(c))
