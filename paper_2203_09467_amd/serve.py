"""Serving loop: events arrive over time and share one device track pool.

An open-loop client of the C ABI.  Events whose arrival time has passed are
submitted to ``transport_events`` together with a bounded number of step
iterations, so requests that arrive while others are on the GPU join the same
pool as soon as event slots, pool room and (if set) the energy budget allow
(continuous batching: admission happens at every host synchronisation inside the
library; a pool that runs full sends its highest-energy tracks to host memory if
the context has spill room); finished events are collected with ``tally_read``
when the library reports some.  Latency of an event = time its tallies were read -
its arrival time.  Results do not depend on the mix: every event's random streams
are keyed by its id and its tallies are fixed-point sums.

A batch refused for lack of event slots or queue room (EMS_E_CAPACITY) is retried
smaller; a stalled pool (EMS_E_STALLED: full of put-off interactions with no spill
room) raises, since its batch was accepted and nothing the loop can do frees room.
"""
from __future__ import annotations

import time
from typing import Dict

import numpy as np

from . import EMS_E_CAPACITY, EMS_NOT_READY, EMS_OK, DeviceEvents, EmsError


def serve(ctx, events, device_events: DeviceEvents = None, iterations: int = 8,
          time_limit: float = 120.0, rate_scale: float = 1.0) -> Dict:
    """Run the arrival schedule ``events.arrival`` (seconds, scaled by 1/rate_scale).

    Returns per-event latency (s), tallies, the track-steps and wall time of the run."""
    dev = device_events or DeviceEvents(events)
    n = events.n_events
    arrival = np.asarray(events.arrival, np.float64) / rate_scale
    latency = np.full(n, np.nan)
    dep = np.zeros((n, ctx.n_bins))
    ledger = np.zeros((n, 5))
    index = {int(e): i for i, e in enumerate(events.event_ids)}
    in_flight = []
    nxt = 0
    max_batch = max(n, 1)  # halved after a refusal for lack of event slots, doubled after a success
    steps = 0
    peak_events = 0
    t0 = time.perf_counter()
    while True:
        now = time.perf_counter() - t0
        if now > time_limit:
            raise RuntimeError(f"serving did not finish within {time_limit} s")
        b = nxt
        while b < n and arrival[b] <= now and b - nxt < max_batch:
            b += 1
        batch = None
        if b > nxt:
            batch = dev.slice(nxt, b)
        if batch is None and not in_flight:
            if nxt >= n:
                break
            time.sleep(max(0.0, min(arrival[nxt] - now, 0.01)))
            continue
        try:
            pr = ctx.transport(batch, iterations)
            if batch is not None:
                in_flight.extend(int(e) for e in batch.ids)
                nxt = b
                max_batch = min(max(n, 1), 2 * max_batch)
        except EmsError as e:  # no free slots or queue room: retry after others finish,
            if e.status != EMS_E_CAPACITY:  # with a smaller batch (a batch is taken whole)
                raise
            max_batch = max(1, (b - nxt) // 2)
            pr = ctx.transport(None, iterations)
        steps += pr.track_steps
        peak_events = max(peak_events, len(in_flight))
        if in_flight and pr.events_done:
            d, L, st = ctx.read(in_flight)
            t_read = time.perf_counter() - t0
            keep = []
            for j, e in enumerate(in_flight):
                if st[j] == EMS_OK:
                    i = index[e]
                    latency[i] = t_read - arrival[i]
                    dep[i] = d[j]
                    ledger[i] = L[j]
                elif st[j] == EMS_NOT_READY:
                    keep.append(e)
                else:
                    raise RuntimeError(f"tally_read status {st[j]} for event {e}")
            in_flight = keep
    wall = time.perf_counter() - t0
    return dict(latency=latency, dep=dep, ledger=ledger, track_steps=steps, wall=wall,
                peak_events=peak_events,
                p50=float(np.percentile(latency, 50)), p99=float(np.percentile(latency, 99)))
