"""The serving loop's scheduling on the CPU, against a model of the library that
needs no GPU: events arrive on a schedule, are submitted when their arrival time
has passed, are refused while the model's event slots are full (EMS_E_CAPACITY,
retried after others finish), and are read back once the model reports finished
events.  Checks that every event is served exactly once, never before it arrives,
that the reported latencies and throughput follow from the schedule, and that a
stalled pool (EMS_E_STALLED) is raised rather than retried as a refusal."""
import types

import numpy as np
import pytest

import paper_2203_09467_amd as ems
from paper_2203_09467_amd.serve import serve


class _Slice:
    def __init__(self, ids):
        self.ids = np.asarray(ids, np.uint32)


class _Device:
    def __init__(self, ids):
        self.ids = np.asarray(ids, np.uint32)

    def slice(self, a, b):
        return _Slice(self.ids[a:b])


class _ModelContext:
    """Each event needs work[e] iterations after admission; at most `slots` events
    are held at once; one iteration takes `dt` seconds of (simulated) device time."""

    def __init__(self, work, slots, n_bins=3):
        self.work = dict(work)
        self.slots = slots
        self.n_bins = n_bins
        self.left = {}
        self.done = set()
        self.read_back = []
        self.refusals = 0

    def transport(self, batch, iterations):
        if batch is not None:
            ids = [int(e) for e in batch.ids]
            if len(self.left) + len(ids) > self.slots:
                self.refusals += 1
                raise ems.EmsError(-3, "transport_events")
            for e in ids:
                assert e not in self.left and e not in self.done
                self.left[e] = self.work[e]
        steps = 0
        for e in list(self.left):
            k = min(iterations, self.left[e])
            self.left[e] -= k
            steps += k
            if self.left[e] == 0:
                del self.left[e]
                self.done.add(e)
        return types.SimpleNamespace(track_steps=steps,
                                     events_done=len(self.done) - len(self.read_back))

    def read(self, ids):
        st = np.array([ems.EMS_OK if int(e) in self.done else ems.EMS_NOT_READY for e in ids],
                      np.int32)
        dep = np.tile(np.arange(self.n_bins, dtype=np.float64), (len(ids), 1)) + np.asarray(ids)[:, None]
        led = np.zeros((len(ids), 5))
        led[:, 0] = np.asarray(ids, np.float64)
        for e, s in zip(ids, st):
            if s == ems.EMS_OK:
                assert int(e) not in self.read_back, "an event was read twice"
                self.read_back.append(int(e))
        return dep, led, st


@pytest.mark.parametrize("slots", [1, 3, 50])
def test_every_event_served_once_after_arrival(slots):
    rng = np.random.default_rng(7)
    n = 40
    ids = np.arange(100, 100 + n, dtype=np.uint32)
    arrival = np.cumsum(rng.exponential(0.002, n))
    events = types.SimpleNamespace(n_events=n, event_ids=ids, arrival=arrival)
    work = {int(e): int(w) for e, w in zip(ids, rng.integers(1, 30, n))}
    ctx = _ModelContext(work, slots)
    res = serve(ctx, events, device_events=_Device(ids), iterations=4, time_limit=30.0)
    assert sorted(ctx.read_back) == sorted(int(e) for e in ids)
    assert np.isfinite(res["latency"]).all() and (res["latency"] >= 0).all()
    assert res["track_steps"] == sum(work.values())
    # tallies land in the row of their event
    assert np.array_equal(res["ledger"][:, 0], ids.astype(np.float64))
    assert np.array_equal(res["dep"][:, 0], ids.astype(np.float64))
    assert res["p50"] <= res["p99"] <= res["latency"].max()
    if slots == 1:
        assert ctx.refusals > 0  # full slots were retried, and nothing was lost
    assert res["peak_events"] >= 1


def test_a_stall_is_not_retried_as_a_refusal():
    class _Stalls(_ModelContext):
        def transport(self, batch, iterations):
            raise ems.EmsError(ems.EMS_E_STALLED, "transport_events")

    ids = np.arange(3, dtype=np.uint32)
    events = types.SimpleNamespace(n_events=3, event_ids=ids, arrival=np.zeros(3))
    ctx = _Stalls({0: 1, 1: 1, 2: 1}, 8)
    with pytest.raises(ems.EmsError) as e:
        serve(ctx, events, device_events=_Device(ids), iterations=4, time_limit=5.0)
    assert e.value.status == ems.EMS_E_STALLED
