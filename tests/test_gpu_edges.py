"""Edge cases of the transport path through the C ABI, against the oracle where a
result is computed: primaries born outside the world, primaries below the tracking
cut (a positron there annihilates at rest), a looper cap of a few steps, empty
and bounded calls, and the error paths (duplicate ids, invalid primaries, too many events,
unknown and unfinished events) that must change no state."""
import dataclasses

import numpy as np
import pytest

import workloads as W
from test_gpu_transport import _ledger_residual, _run_gpu

pytestmark = pytest.mark.gpu


def _events(species, energy, pos, dirs, ids=None):
    n = len(species)
    ids = np.arange(n, dtype=np.uint32) if ids is None else np.asarray(ids, np.uint32)
    return W.Events(ids, np.arange(n + 1, dtype=np.int64), np.asarray(species, np.int32),
                    np.asarray(energy, np.float64), np.asarray(pos, np.float64).reshape(n, 3),
                    np.asarray(dirs, np.float64).reshape(n, 3))


def _context(wl, max_events=64, pool=1 << 16):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=pool, max_events=max_events, max_bins=wl.geometry.n_bins,
                      queue_capacity=1024, seed=wl.seed)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    return ctx


def _match_oracle(orc, wl, ev, g):
    o = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, ev)
    e_in = o["ledger"][:, 0]
    assert np.array_equal(g["ledger"][:, 0], e_in)
    assert np.abs(_ledger_residual(g["dep"], g["ledger"])).max() < 1e-12
    assert (np.abs(g["dep"] - o["dep"]).max(1) <= 1e-9 * e_in).all()
    assert (np.abs(g["ledger"][:, 1:3] - o["ledger"][:, 1:3]).max(1) <= 1e-9 * e_in).all()
    assert np.array_equal(g["ledger"][:, 3:], o["ledger"][:, 3:])
    return o


def test_outside_and_below_cut_primaries(orc):
    wl = W.calorimeter(1)
    ev = _events(species=[W.ELECTRON, W.GAMMA, W.ELECTRON, W.POSITRON, W.GAMMA, W.POSITRON],
                 energy=[100.0, 50.0, 0.005, 0.005, 0.5, 30.0],
                 pos=[[0, 0, -10], [100, 0, 5], [0, 0, 1.0], [0, 0, 1.0], [0, 0, 0], [3, -2, 0]],
                 dirs=[[0, 0, 1]] * 6)
    g = _run_gpu(wl, ev)
    _match_oracle(orc, wl, ev, g)
    # born outside: escapes with its whole energy, deposits nothing
    assert g["ledger"][0, 1] == 100.0 and g["ledger"][1, 1] == 50.0
    assert g["dep"][0].sum() == 0.0 and g["dep"][1].sum() == 0.0
    # below the tracking cut: deposited at once; the positron also annihilates at rest
    assert abs(g["dep"][2].sum() - 0.005) <= 1e-15
    assert g["ledger"][3, 4] == 1


def test_looper_cap_of_three_steps(orc):
    wl = W.calorimeter(30)
    wl = dataclasses.replace(wl, options=dataclasses.replace(wl.options, max_steps=3))
    g = _run_gpu(wl, wl.events)
    _match_oracle(orc, wl, wl.events, g)
    assert (g["ledger"][:, 2] > 0).all()  # every 1 GeV shower was cut short: energy killed


def test_empty_and_bounded_calls():
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(4, energy=10_000.0)
    ctx = _context(wl)
    pr = ctx.transport(None, -1)
    assert pr.alive == 0 and pr.track_steps == 0 and pr.queued_events == 0
    dev = ems.DeviceEvents(wl.events)
    pr = ctx.transport(dev, 0)  # submitted, not yet stepped
    assert pr.track_steps == 0 and pr.queued_events == 4
    pr = ctx.transport(None, 2)
    assert pr.track_steps > 0 and pr.alive > 0
    _, _, status = ctx.read(wl.events.event_ids)
    assert (status == ems.EMS_NOT_READY).all()
    pr = ctx.transport(None, -1)
    assert pr.alive == 0
    dep, led, status = ctx.read(wl.events.event_ids)
    assert (status == ems.EMS_OK).all()
    assert np.abs(_ledger_residual(dep, led)).max() < 1e-12
    # a finished event's slot is released by the read: its id is unknown afterwards
    _, _, status = ctx.read(wl.events.event_ids[:1])
    assert status[0] == -1


def test_error_paths_change_no_state():
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(3)
    ctx = _context(wl, max_events=8)
    dup = _events([W.ELECTRON] * 2, [1000.0] * 2, [[0, 0, 0]] * 2, [[0, 0, 1]] * 2, ids=[7, 7])
    with pytest.raises(ems.EmsError) as e:
        ctx.transport(ems.DeviceEvents(dup), -1)
    assert e.value.status == -1
    bad = _events([5], [1000.0], [[0, 0, 0]], [[0, 0, 1]], ids=[9])
    with pytest.raises(ems.EmsError) as e:
        ctx.transport(ems.DeviceEvents(bad), -1)
    assert e.value.status == -1
    for sp, T, pos, d in ((W.GAMMA, 0.0, [0, 0, 0], [0, 0, 1]),            # no energy
                          (W.ELECTRON, np.nan, [0, 0, 0], [0, 0, 1]),       # energy not finite
                          (W.ELECTRON, 2.0e5, [0, 0, 0], [0, 0, 1]),        # above the tables
                          (W.GAMMA, 10.0, [np.inf, 0, 0], [0, 0, 1]),       # position not finite
                          (W.GAMMA, 10.0, [0, 0, 0], [0, 0.5, 0.5])):       # not a unit vector
        with pytest.raises(ems.EmsError) as e:
            ctx.transport(ems.DeviceEvents(_events([sp], [T], [pos], [d], ids=[11])), -1)
        assert e.value.status == -1
    too_many = _events([W.ELECTRON] * 9, [1.0] * 9, [[0, 0, 0]] * 9, [[0, 0, 1]] * 9,
                       ids=np.arange(20, 29))
    with pytest.raises(ems.EmsError) as e:
        ctx.transport(ems.DeviceEvents(too_many), -1)
    assert e.value.status == -3
    _, _, status = ctx.read(np.array([7, 9, 11, 20, 12345], np.uint32))
    assert (status == -1).all()  # none of them was submitted
    # the context still works and gives the same tallies as a fresh one
    pr = ctx.transport(ems.DeviceEvents(wl.events), -1)
    assert pr.alive == 0
    dep, led, status = ctx.read(wl.events.event_ids)
    ref = _run_gpu(wl, wl.events)
    assert (status == 0).all() and np.array_equal(dep, ref["dep"]) and np.array_equal(led, ref["ledger"])
