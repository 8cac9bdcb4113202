"""Serving loop: Poisson arrivals share one device pool (continuous batching); every
event's tallies are bitwise the same when it is transported alone."""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
ME = 0.51099895


def _context(wl, n_events, precision=0, pool=1 << 22, budget=2.0e7):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=pool, max_events=n_events, max_bins=wl.geometry.n_bins,
                      queue_capacity=max(wl.events.n_primaries, 1), seed=wl.seed,
                      precision=precision, energy_budget=budget, iterations_per_sync=4)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    return ctx


@pytest.mark.parametrize("precision", [0, 1])
def test_serving_alone_equals_mix(precision):
    import paper_2203_09467_amd as ems
    from paper_2203_09467_amd.serve import serve
    wl = W.serving(n_events=24, rate_hz=300.0)
    ev = wl.events
    ev.energy[:] *= 0.05  # 50 MeV - 5 GeV primaries keep the test short
    ctx = _context(wl, ev.n_events, precision)
    res = serve(ctx, ev, iterations=4, time_limit=100.0)
    assert np.isfinite(res["latency"]).all()
    L = res["ledger"]
    bal = L[:, 0] - (res["dep"].sum(1) + L[:, 1] + L[:, 2] + 2 * ME * (L[:, 3] - L[:, 4]))
    assert np.abs(bal / L[:, 0]).max() < 1e-12
    assert res["peak_events"] >= 2  # events overlapped on the device
    for i in (0, 7, 23):
        alone = _context(wl, 1, precision)
        one = ev.subset([i])
        alone.transport(ems.DeviceEvents(one), -1)
        d, led, st = alone.read(one.event_ids)
        assert st[0] == 0
        assert np.array_equal(d[0], res["dep"][i])
        assert np.array_equal(led[0], res["ledger"][i])
