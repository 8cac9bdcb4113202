"""Paths of the transport library that only unusual sizes reach, through the C ABI:

* the global-memory variant of the step kernels (run data too large to stage in
  LDS: six materials in FP64), single-step and event parity with the oracle;
* a pool too small for a shower: without host memory to spill to, the library
  reports EMS_E_STALLED (every kernel exits normally: the stall is detected by
  the interaction kernel's room check); with spill room it completes, moving the
  tracks of highest energy to host memory, and every event's tallies are bitwise
  those of a pool large enough never to spill;
* per-event track-steps by species and per-event escape spectra from tally_read,
  against the oracle run one event at a time;
* a read that names one id twice returns it once and releases its slot once.
"""
import numpy as np
import pytest

import workloads as W
from test_gpu_step_parity import _compare, _ctx_for, _states
from test_gpu_transport import _ledger_residual, _run_gpu

pytestmark = pytest.mark.gpu

STAGE_BUDGET = 64 * 1024  # bytes of run data a step-kernel block stages in LDS


def test_unstaged_kernels_six_materials(orc):
    wl = W.material_stack(120)
    tab_bytes = len(wl.materials) * 2 * 200 * 4 * 8  # charged tables of every material, FP64
    assert tab_bytes > STAGE_BUDGET
    w = orc.World(wl.materials, wl.options, wl.geometry)
    n = 8000
    st = _states(wl, n, 606)
    ctx = _ctx_for(wl, n)
    records, out = ctx.step_once(st)
    bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"
    ctx.close()
    g = _run_gpu(wl, wl.events)
    o = w.run_events(wl.seed, wl.events)
    e_in = o["ledger"][:, 0]
    assert np.abs(_ledger_residual(g["dep"], g["ledger"])).max() < 1e-12
    match = (np.abs(g["dep"] - o["dep"]).max(1) <= 1e-9 * e_in).mean()
    assert match >= 0.97, match


def _small_pool_context(wl, pool, spill):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=pool, max_events=wl.events.n_events, max_bins=wl.geometry.n_bins,
                      queue_capacity=wl.events.n_primaries, seed=wl.seed, spill_capacity=spill,
                      iterations_per_sync=4)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    return ctx


def test_stall_without_spill_room():
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(4, energy=10_000.0)
    ctx = _small_pool_context(wl, 64, 0)
    with pytest.raises(ems.EmsError) as e:
        ctx.transport(ems.DeviceEvents(wl.events), 4000)
    assert e.value.status == ems.EMS_E_STALLED
    # the batch stays accepted: its events are in flight, not unknown
    _, _, status = ctx.read(wl.events.event_ids)
    assert (status == ems.EMS_NOT_READY).all()
    ctx.close()


def test_spill_to_host_memory_changes_no_result():
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(8, energy=10_000.0)
    ref = _run_gpu(wl, wl.events)
    ctx = _small_pool_context(wl, 1024, 1 << 20)
    pr = ctx.transport(ems.DeviceEvents(wl.events), -1)
    assert pr.alive == 0 and pr.spilled == 0
    assert pr.spilled_total > 0  # the showers did not fit: tracks waited in host memory
    assert pr.peak_alive <= 1024
    dep, led, status = ctx.read(wl.events.event_ids)
    assert (status == 0).all()
    assert np.array_equal(dep, ref["dep"]) and np.array_equal(led, ref["ledger"])


def test_per_event_steps_and_escape_spectra(orc):
    import paper_2203_09467_amd as ems
    w_cal = W.calorimeter(12)
    w_cube = W.photon_cube(300)
    for wl in (w_cal, w_cube):
        ne = wl.events.n_events
        ctx = ems.Context(pool_capacity=1 << 20, max_events=ne, max_bins=wl.geometry.n_bins,
                          queue_capacity=wl.events.n_primaries, seed=wl.seed, event_escape=True)
        ctx.setup(wl.materials, wl.options, wl.geometry)
        ctx.transport(ems.DeviceEvents(wl.events), -1)
        run_steps, run_hist = ctx.counters()
        dep, led, status, steps, esc = ctx.read(wl.events.event_ids, steps=True, escape=True)
        assert (status == 0).all()
        # the per-event figures add up to the run's
        assert np.array_equal(steps.sum(0), run_steps)
        assert np.array_equal(esc.sum(0), run_hist)
        w = orc.World(wl.materials, wl.options, wl.geometry)
        n_equal = 0
        for i in range(ne):
            o = w.run_events(wl.seed, wl.events.subset([i]), esc_hist=True)
            if np.abs(dep[i] - o["dep"][0]).max() > 1e-9 * led[i, 0]:
                continue  # a rounding difference sent this history elsewhere
            n_equal += 1
            assert np.array_equal(steps[i], o["steps"]), i
            assert np.array_equal(esc[i], o["esc_hist"].astype(np.uint64)), i
        assert n_equal >= 0.9 * ne
        ctx.close()


def test_escape_spectra_need_the_flag():
    import paper_2203_09467_amd as ems
    wl = W.photon_cube(4)
    ctx = ems.Context(pool_capacity=1 << 12, max_events=4, max_bins=1, queue_capacity=4,
                      seed=wl.seed)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    ctx.transport(ems.DeviceEvents(wl.events), -1)
    with pytest.raises(ems.EmsError) as e:
        ctx.read(wl.events.event_ids, escape=True)
    assert e.value.status == ems.EMS_E_STATE
    _, _, status = ctx.read(wl.events.event_ids)  # nothing was released by the refused call
    assert (status == 0).all()


def test_repeated_id_is_read_once():
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(4)
    ctx = ems.Context(pool_capacity=1 << 16, max_events=4, max_bins=wl.geometry.n_bins,
                      queue_capacity=64, seed=wl.seed)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    ctx.transport(ems.DeviceEvents(wl.events.subset([0, 1])), -1)
    ids = wl.events.event_ids
    dep, led, status = ctx.read(np.array([ids[0], ids[0], ids[1]], np.uint32))
    assert list(status) == [0, ems.EMS_E_ARG, 0]
    assert np.array_equal(dep[1], np.zeros_like(dep[1]))
    # the slots came back once each: two more events fit the four slots with two to spare
    ctx.transport(ems.DeviceEvents(wl.events.subset([2, 3])), -1)
    extra = W.calorimeter(2, first_id=100)
    ctx.transport(ems.DeviceEvents(extra.events), -1)
    d2, l2, s2 = ctx.read(np.concatenate([ids[2:4], extra.events.event_ids]))
    assert (s2 == 0).all()
    ref = _run_gpu(wl, wl.events)
    assert np.array_equal(d2[:2], ref["dep"][2:4]) and np.array_equal(l2[:2], ref["ledger"][2:4])
    assert np.array_equal(dep[0], ref["dep"][0]) and np.array_equal(dep[2], ref["dep"][1])


def test_iteration_log():
    """Per-iteration records: one per busy iteration, pool sizes chaining from one
    iteration's output to the next one's input, totals equal to the run statistics."""
    import paper_2203_09467_amd as ems
    wl = W.calorimeter(40)
    ctx = ems.Context(pool_capacity=1 << 18, max_events=40, max_bins=wl.geometry.n_bins,
                      queue_capacity=64, seed=wl.seed, time_steps=True, iterations_per_sync=4)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    ctx.step_stats(reset=True)
    pr = ctx.transport(ems.DeviceEvents(wl.events), -1)
    st = ctx.step_stats()
    log = ctx.iteration_log(reset=True)
    assert len(log) == pr.iterations == st.launches
    n_in = log["photons"].astype(np.int64) + log["charged"]
    assert n_in.sum() == st.tracks_in
    assert log["tracks_out"][-1] == 0
    # with every event admitted at the start, each iteration takes the previous one's output
    assert np.array_equal(n_in[1:], log["tracks_out"][:-1].astype(np.int64))
    # iterations of the last sync interval that found the pool empty are timed but
    # not recorded; they take a few microseconds each
    assert (log["ms"] > 0).all()
    assert log["ms"].sum() <= st.kernel_ms * (1 + 1e-6) and log["ms"].sum() >= 0.98 * st.kernel_ms
    assert int(n_in.max()) == pr.peak_alive
    assert len(ctx.iteration_log()) == 0  # the reset cleared it
