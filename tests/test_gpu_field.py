"""Barrel geometry in a uniform 1 T field: the HIP step (RK4 substeps with
step-doubling error control, chord boundary search) against the oracle's, and
barrel events event by event (FP64).  Tolerances as in test_gpu_step_parity."""
import numpy as np
import pytest

import workloads as W
from test_gpu_step_parity import _compare

pytestmark = pytest.mark.gpu
ME = 0.51099895


def _ctx(wl, n, precision=0):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=max(4 * n, 4096), max_events=max(n, 1),
                      max_bins=wl.geometry.n_bins, queue_capacity=4096, seed=wl.seed,
                      precision=precision)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    return ctx


@pytest.mark.parametrize("n,seed,e_lo", [(6000, 21, 0.01), (3000, 22, 1.0)])
def test_barrel_step_parity(orc, n, seed, e_lo):
    wl = W.barrel(1)
    g = wl.geometry
    st = W.random_track_states(n, g.n_vol, seed, e_lo=e_lo, bounds=g.bounds, kind=1,
                               half_z=g.half_z)
    st["event"] = np.zeros(n, np.uint32)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    records, out = _ctx(wl, n).step_once(st)
    ores = w.step_tracks(wl.seed, st)
    bad = _compare(wl, st, records, out, ores)
    detail = [(i, int(st["species"][i]), float(st["energy"][i]), int(st["vol"][i]),
               (ores[i].limiter, ores[i].step_len, ores[i].n_out),
               (int(records[i]["limiter"]), float(records[i]["step_len"]), int(records[i]["n_out"])))
              for i in bad[:4]]
    assert not bad, f"{len(bad)} of {n} states differ: {detail}"
    charged = st["species"] != 0
    assert (records["limiter"][charged] == 0).any() and (records["limiter"][charged] == 1).any()


def test_barrel_events(orc):
    import paper_2203_09467_amd as ems
    wl = W.barrel(24)
    ev = wl.events
    ev.energy[:] = np.random.default_rng(3).uniform(500.0, 3000.0, ev.n_events)
    ctx = ems.Context(pool_capacity=1 << 20, max_events=ev.n_events, max_bins=wl.geometry.n_bins,
                      queue_capacity=ev.n_primaries, seed=wl.seed)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    ctx.transport(ems.DeviceEvents(ev), -1)
    dep, led, status = ctx.read(ev.event_ids)
    assert (status == 0).all()
    bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * ME * (led[:, 3] - led[:, 4]))
    assert np.abs(bal / led[:, 0]).max() < 1e-12
    o = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, ev)
    match = np.abs(dep - o["dep"]).max(1) <= 1e-9 * led[:, 0]
    assert match.mean() >= 0.9, match.mean()


def test_vacuum_steps_on_their_substep_cap(orc):
    """Low-momentum e-/e+ in the barrel's vacuum regions: a field step in vacuum ends
    after 256 substeps (limiter 4, the count of such steps in a row carried with the
    track) and the 40th in a row kills the track as a looper (limiter 3)."""
    wl = W.barrel(1)
    g = wl.geometry
    n = 4000
    st = W.random_track_states(n, g.n_vol, 31, e_lo=0.01, e_hi=2.0, bounds=g.bounds, kind=1,
                               half_z=g.half_z)
    vac = np.where(g.material < 0)[0]
    rng = np.random.default_rng(32)
    st["vol"] = rng.choice(vac, n).astype(np.int32)
    lo, hi = g.bounds[st["vol"]], g.bounds[st["vol"] + 1]
    r = lo + (hi - lo) * rng.random(n)
    a = 2 * np.pi * rng.random(n)
    st["pos"][:, 0], st["pos"][:, 1] = r * np.cos(a), r * np.sin(a)
    st["species"] = rng.integers(1, 3, n).astype(np.int32)
    st["vcap"] = rng.integers(0, 40, n).astype(np.uint32)
    st["event"] = np.zeros(n, np.uint32)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    records, out = _ctx(wl, n).step_once(st)
    bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"
    lim = set(np.unique(records["limiter"]))
    assert {3, 4} <= lim


def _barrel_run(wl, ev, field_substeps, pool=1 << 20, spill=0):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=pool, max_events=ev.n_events, max_bins=wl.geometry.n_bins,
                      queue_capacity=ev.n_primaries, seed=wl.seed, spill_capacity=spill,
                      field_substeps=field_substeps)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    pr = ctx.transport(ems.DeviceEvents(ev), -1)
    dep, led, status = ctx.read(ev.event_ids)
    assert (status == 0).all()
    steps, _, life = ctx.counters(life=True)
    ctx.close()
    return dep, led, steps, life, pr


def test_suspended_curved_moves_change_no_result():
    """A curved move that runs out of its launch's substeps is suspended and continued
    by the next launch where it stood: with 1 substep per step (nearly every move
    suspended, many times), the default, and 1024 (almost none), every event's
    tallies, ledger, step counts and steps-per-track histogram are bitwise the same;
    so they are with a small pool that spills suspended moves to host memory."""
    wl = W.barrel(16)
    ev = wl.events
    ev.energy[:] = np.random.default_rng(5).uniform(200.0, 2000.0, ev.n_events)
    ref = _barrel_run(wl, ev, 1024)
    for fs, pool, spill in ((1, 1 << 20, 0), (0, 1 << 20, 0), (2, 1 << 9, 1 << 20)):
        got = _barrel_run(wl, ev, fs, pool, spill)
        for a, b in zip(ref[:4], got[:4]):
            assert np.array_equal(a, b), (fs, pool)
        if spill:
            assert got[4].spilled_total > 0
    assert ref[4].iterations < _barrel_run(wl, ev, 1)[4].iterations
