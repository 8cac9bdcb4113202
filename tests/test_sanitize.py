"""Sanitizer builds on the CPU (no GPU): the oracle compiled with AddressSanitizer and
UndefinedBehaviorSanitizer transports events of every geometry kind and steps random
states, and the library's event bookkeeping -- the id -> slot table its kernels probe
and the per-batch admission queue of its host side -- is fuzzed against plain
references under the same sanitizers.  Any sanitizer report fails the test."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SAN = ["-fsanitize=address,undefined", "-fno-sanitize-recover=all", "-fno-omit-frame-pointer", "-g",
       "-O1"]


def _libasan():
    r = subprocess.run(["gcc", "-print-file-name=libasan.so"], capture_output=True, text=True)
    path = r.stdout.strip()
    if r.returncode != 0 or not os.path.isabs(path) or not os.path.exists(path):
        pytest.skip("no AddressSanitizer runtime for gcc")
    return path


def test_event_bookkeeping_under_sanitizers(tmp_path):
    _libasan()
    exe = tmp_path / "slots_fuzz"
    subprocess.run(["g++", "-std=c++17", *SAN, "-I", os.path.join(ROOT, "paper_2203_09467_amd", "csrc"),
                    os.path.join(ROOT, "tests", "sanitize", "slots_fuzz.cpp"), "-o", str(exe)], check=True)
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300)
    assert r.returncode == 0, r.stdout + r.stderr
    assert "slots ok" in r.stdout


_DRIVER = r"""
import sys
import numpy as np
sys.path.insert(0, sys.argv[1])
import oracle
oracle.LIB_PATH = sys.argv[2]
import workloads as W
for wl, n in ((W.photon_cube(60), None), (W.calorimeter(6), None), (W.calorimeter(4, energy=10000.0), None),
              (W.barrel(3), None), (W.csg_module(8), None), (W.material_stack(3), None)):
    w = oracle.World(wl.materials, wl.options, wl.geometry)
    r = w.run_events(wl.seed, wl.events, esc_hist=True)
    assert np.isfinite(r["dep"]).all()
wl = W.calorimeter(1)
w = oracle.World(wl.materials, wl.options, wl.geometry)
st = W.random_track_states(3000, wl.geometry.n_vol, 3, bounds=wl.geometry.bounds)
st["event"] = np.zeros(3000, np.uint32)
w.step_tracks(wl.seed, st)
print("oracle ok")
"""


def test_oracle_under_sanitizers(tmp_path):
    libasan = _libasan()
    lib = tmp_path / "liboracle_san.so"
    src = [os.path.join(ROOT, "oracle", f) for f in ("philox.c", "physics.c", "transport.c", "field.c",
                                                     "csg.c")]
    subprocess.run(["gcc", "-std=c99", *SAN, "-ffp-contract=off", "-fPIC", "-shared", "-o", str(lib),
                    *src, "-lm"], check=True)
    env = dict(os.environ, LD_PRELOAD=libasan, ASAN_OPTIONS="detect_leaks=0",
               UBSAN_OPTIONS="print_stacktrace=1")
    r = subprocess.run([sys.executable, "-c", _DRIVER, ROOT, str(lib)], capture_output=True, text=True,
                       timeout=600, env=env)
    assert r.returncode == 0, r.stderr[-4000:]
    assert "oracle ok" in r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr
