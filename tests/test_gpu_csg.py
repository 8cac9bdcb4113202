"""Quadric-surface cell navigation on the GPU, through the C ABI.

* Single-step parity with the oracle in the module of spheres, an x-cylinder, a
  cone and planes (random states inside cells, and states sitting exactly on the
  boundary point where the oracle's previous straight step crossed into a cell),
  at the 1e-12 bar of the other single-step tests.
* The slab calorimeter written as quadric cells gives, on the GPU, bitwise the
  tallies of the slab navigation.
* Module events against the oracle: events equal to 1e-9 E_in, per-cell sums
  within 3 sigma + 0.1 %, energy conserved to 1e-12.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_step_parity import _compare, _ctx_for
from test_gpu_transport import _layer_check, _ledger_residual, _run_gpu

pytestmark = pytest.mark.gpu


def _module_states(w, n, seed):
    rng = np.random.default_rng(seed)
    pos, dirs, vols = [], [], []
    while len(vols) < n:
        p = rng.uniform(-20, 20, 3)
        c = 2 * rng.random() - 1
        ph = 2 * np.pi * rng.random()
        s = np.sqrt(1 - c * c)
        d = np.array([s * np.cos(ph), s * np.sin(ph), c])
        k = w.locate(p, d)
        if k < 0:
            continue
        if rng.random() < 0.3:  # move to where the straight ray enters the next cell
            t, nxt = w.distance(k, p, d)
            if nxt < 0:
                continue
            p = p + t * d
            k = nxt
        pos.append(p)
        dirs.append(d)
        vols.append(k)
    sp = rng.integers(0, 3, n).astype(np.int32)
    T = np.exp(np.log(0.01) + rng.random(n) * np.log(1e7))
    nlam = np.where(rng.random(n) < 0.5, -1.0, rng.exponential(1.0, n))
    key = rng.integers(0, 2 ** 32, size=(n, 3), dtype=np.uint64).astype(np.uint32)
    nstep = rng.integers(0, 1000, n).astype(np.uint32)
    return dict(species=sp, energy=T, vol=np.array(vols, np.int32), pos=np.array(pos),
                dir=np.array(dirs), nlam=nlam, key=key, nstep=nstep,
                event=np.zeros(n, np.uint32))


def test_module_step_parity(orc):
    wl = W.csg_module(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    n = 12000
    st = _module_states(w, n, 77)
    ctx = _ctx_for(wl, n)
    records, out = ctx.step_once(st)
    bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"
    assert set(np.unique(records["limiter"])) >= {0, 1, 2}


def test_calorimeter_as_cells_equals_slabs():
    wl = W.calorimeter(300)
    slab = _run_gpu(wl, wl.events)
    csg = W.Workload(wl.name, wl.materials, wl.options, W.calorimeter_csg(), wl.events, wl.seed)
    cells = _run_gpu(csg, wl.events)
    assert np.array_equal(slab["dep"], cells["dep"])
    assert np.array_equal(slab["ledger"], cells["ledger"])
    assert np.array_equal(slab["steps"], cells["steps"])


def test_module_events_against_oracle(orc):
    wl = W.csg_module(600)
    g = _run_gpu(wl, wl.events)
    o = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, wl.events)
    e_in = o["ledger"][:, 0]
    assert np.array_equal(g["ledger"][:, 0], e_in)
    assert np.abs(_ledger_residual(g["dep"], g["ledger"])).max() < 1e-12
    match = (np.abs(g["dep"] - o["dep"]).max(1) <= 1e-9 * e_in).mean()
    assert match >= 0.97, match
    assert _layer_check(g["dep"], o["dep"]).all()
