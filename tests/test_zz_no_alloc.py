"""The entry point that allocates nothing: ems_create_static builds a context over the
library's static device scratch instead of a caller workspace.  Two contexts in a
row on the same scratch -- the second with a smaller batch, over memory the first
one left behind -- give bitwise the tallies of contexts over torch workspaces."""
import ctypes as C

import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu


def _create_static(cfg):
    import paper_2203_09467_amd as ems
    h = C.c_void_p()
    return ems._lib.ems_create_static(C.byref(cfg), C.byref(h)), h


def _run(h, wl, events, n_bins):
    import paper_2203_09467_amd as ems
    ems.init_physics_tables(h, wl.materials, wl.options)
    ems.init_geometry(h, wl.geometry)
    pr = ems.transport_events(h, ems.DeviceEvents(events), -1)
    assert pr.alive == 0
    dep, led, status, steps = ems.tally_read(h, events.event_ids, n_bins, steps=True)
    assert (status == 0).all()
    return dep, led, steps


def _reference(wl, events, cfg):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=cfg.pool_capacity, max_events=cfg.max_events,
                      max_bins=cfg.max_bins, queue_capacity=cfg.queue_capacity, seed=cfg.seed)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    ctx.transport(ems.DeviceEvents(events), -1)
    dep, led, status, steps = ctx.read(events.event_ids, steps=True)
    assert (status == 0).all()
    ctx.close()
    return dep, led, steps


def test_static_context_twice_equals_workspace_context():
    import paper_2203_09467_amd as ems
    big = W.calorimeter(40)
    small = W.calorimeter(12, energy=3000.0, first_id=500)
    for wl in (big, small):
        ev = wl.events
        cfg = ems.Config(1 << 17, 64, wl.geometry.n_bins, 4096, wl.seed, ems.EMS_FP64, 0.0, 0, 0, 0)
        st, h = _create_static(cfg)
        assert st == 0, ems._lib.ems_last_error()
        try:
            got = _run(h, wl, ev, wl.geometry.n_bins)
        finally:
            ems._lib.ems_destroy(h)
        ref = _reference(wl, ev, cfg)
        for a, b in zip(got, ref):
            assert np.array_equal(a, b)


def test_static_context_limits():
    import paper_2203_09467_amd as ems
    too_big = ems.Config(1 << 22, 64, 100, 4096, 1, ems.EMS_FP64, 0.0, 0, 0, 0)
    st, _ = _create_static(too_big)
    assert st == ems.EMS_E_CAPACITY
    assert b"static scratch" in ems._lib.ems_last_error()
    timed = ems.Config(1 << 12, 8, 100, 64, 1, ems.EMS_FP64, 0.0, ems.EMS_FLAG_TIME_STEPS, 0, 0)
    st, _ = _create_static(timed)
    assert st == ems.EMS_E_ARG
