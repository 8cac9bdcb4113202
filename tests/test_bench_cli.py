"""bench.py's command-line contract on the CPU: a request for more than one GPU
exits with a message (this build runs on one GPU), and the measured-traffic lookup
applies only to the workload and settings it was measured with."""
import importlib.util
import json
import os
import subprocess
import sys
import types

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


def test_traffic_applies_only_to_its_settings():
    b = _bench()
    with open(b.TRAFFIC_FILE) as f:
        t = json.load(f)
    base = dict(precision="fp64", events=100_000, energy=1000.0, budget=t["energy_budget_MeV"],
                pool=t["pool_slots"], per_sync=t["iterations_per_sync"])
    assert b.measured_traffic(types.SimpleNamespace(**base)) == t["bytes_per_iteration"]
    for k, v in (("precision", "mixed"), ("events", 1000), ("budget", 1.0), ("per_sync", 1)):
        assert b.measured_traffic(types.SimpleNamespace(**{**base, k: v})) is None


def test_kernel_digest_ignores_comments(tmp_path):
    b = _bench()
    a = tmp_path / "a.hip"
    c = tmp_path / "b.hip"
    a.write_text("int f() { return 1; }  // one\n/* block */\n")
    c.write_text("int f()   {\n  return 1;\n}\n")
    assert b.kernel_source_digest(str(a)) == b.kernel_source_digest(str(c))
    c.write_text("int f() { return 2; }\n")
    assert b.kernel_source_digest(str(a)) != b.kernel_source_digest(str(c))
