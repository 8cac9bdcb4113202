"""Benchmark: electromagnetic-shower transport throughput on one MI355X.

Workload (default): 1e5 primary 1 GeV electrons at normal incidence on the
50-layer 2 mm Pb + 5 mm LAr calorimeter (40 x 40 cm), full e-/e+/photon physics,
0.7 mm production cut, FP64, seed 2.  One benchmark "step" is the transport of
the whole batch to completion (every step of the hot path: admission, cross
sections, interaction lengths, step limits, boundaries, continuous loss,
interactions, secondaries, compaction, tallies) with the primaries already
resident in HBM.  value = track-steps / s over the timed steps.

Also reported: the step kernel against the HBM roofline (algorithmic bytes =
88 B read per track in the pool + 88 B written per surviving track or secondary,
divided by the step kernels' summed HIP-event durations on their launch stream),
and the CPU oracle timed on a bounded sample of the same workload on the host
cores (cpu_baseline).
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
BYTES_PER_TRACK = 88  # SoA state of one track: 8 doubles + 6 words


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def _oracle_worker(args):
    seed, lo, hi, n_events, energy = args
    import oracle
    import workloads as W
    wl = W.calorimeter(n_events, energy=energy, seed=seed)
    w = oracle.World(wl.materials, wl.options, wl.geometry)
    ev = wl.events.subset(np.arange(lo, hi))
    t0 = time.perf_counter()
    r = w.run_events(wl.seed, ev)
    return int(r["steps"].sum()), time.perf_counter() - t0


def cpu_baseline(n_events, energy, seed, budget_s=12.0):
    """The oracle as it stands, events split across processes on the host cores."""
    import multiprocessing as mp
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    cores = max(1, min(cores, 16))
    # calibrate on a few events, then size the sample for ~budget_s of wall time
    steps, dt = _oracle_worker((seed, 0, 20, n_events, energy))
    rate1 = steps / max(dt, 1e-9)
    per_event = steps / 20
    n_sample = int(min(n_events, max(cores * 20, rate1 * budget_s * cores / per_event)))
    chunks = np.linspace(0, n_sample, cores + 1).astype(int)
    jobs = [(seed, int(a), int(b), n_events, energy) for a, b in zip(chunks[:-1], chunks[1:]) if b > a]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    return dict(value=total / wall, unit="track-steps/s", cores=len(jobs), kind="oracle",
                sample=f"events 0..{n_sample - 1} of the benchmark batch ({total} track-steps, "
                       f"{wall:.1f} s wall, {len(jobs)} processes)")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=100_000)
    ap.add_argument("--energy", type=float, default=1000.0, help="primary energy, MeV")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--pool", type=int, default=1 << 24)
    ap.add_argument("--budget", type=float, default=2.5e7, help="energy in flight, MeV")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) three times, "
                         "to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1"}))
        sys.exit(2)
    if args.copy_calibration:
        import torch
        n = args.copy_calibration * (1 << 20) // 4
        src = torch.ones(n, dtype=torch.float32, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            torch.mul(src, 1.0, out=dst)
        torch.cuda.synchronize()
        print(json.dumps({"copy_calibration_bytes_read": n * 4, "bytes_written": n * 4,
                          "launches": 3}))
        return

    import torch

    import paper_2203_09467_amd as ems
    import workloads as W

    seed = 2
    wl = W.calorimeter(args.events, energy=args.energy, seed=seed)
    n_steps = args.warmup + args.steps
    prec = ems.EMS_FP64 if args.precision == "fp64" else ems.EMS_MIXED
    ctx = ems.Context(pool_capacity=args.pool, max_events=args.events * n_steps,
                      max_bins=wl.geometry.n_bins, queue_capacity=args.events, seed=seed,
                      precision=prec, energy_budget=args.budget, time_steps=True)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    batches = []
    for j in range(n_steps):
        ev = wl.events.subset(np.arange(args.events))
        ev.event_ids = (np.arange(args.events) + j * args.events).astype(np.uint32)
        batches.append(ems.DeviceEvents(ev))
    torch.cuda.synchronize()

    total_steps = 0
    t_run = 0.0
    iters = 0
    peak = 0
    for j in range(n_steps):
        timed = j >= args.warmup
        if timed and j == args.warmup:
            ctx.step_stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        ts = time.perf_counter()
        pr = ctx.transport(batches[j], -1)
        torch.cuda.synchronize()
        dt = time.perf_counter() - ts
        log(f"step {j} ({'timed' if timed else 'warmup'}): {pr.track_steps} track-steps in "
            f"{dt:.3f} s, {pr.iterations} iterations, peak pool {pr.peak_alive}, "
            f"deferred {pr.deferred}")
        if timed:
            total_steps += pr.track_steps
            iters += pr.iterations
            peak = max(peak, pr.peak_alive)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    st = ctx.step_stats()

    # correctness of what was timed: every event conserves energy
    ids = np.concatenate([b.ids for b in batches[args.warmup:]])
    dep, led, status = ctx.read(ids)
    assert (status == 0).all()
    bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * 0.51099895 * (led[:, 3] - led[:, 4]))
    ledger_max = float(np.abs(bal / led[:, 0]).max())

    value = total_steps / t_run
    bytes_alg = BYTES_PER_TRACK * (st.tracks_in + st.tracks_out)
    kernel_s = st.kernel_ms / 1e3
    achieved = bytes_alg / kernel_s / 1e9 if kernel_s > 0 else 0.0
    out = {
        "metric": "track-steps/s (FP64 vs mixed-prec) + p50/p99 event latency, 1 MI355X",
        "value": value,
        "unit": "track-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": t_run / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == ems.EMS_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"calorimeter: {args.events} x {args.energy / 1000:g} GeV e- on "
                               "50 x (2 mm Pb + 5 mm LAr), 40x40 cm, 0.7 mm cut, seed 2",
                   "precision": args.precision, "pool_slots": args.pool,
                   "energy_budget_MeV": args.budget, "iterations": iters,
                   "peak_tracks_in_flight": peak, "track_steps": total_steps,
                   "ledger_max_rel_error": ledger_max},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "k_step<double>" if prec == ems.EMS_FP64 else "k_step<float>",
                     "launches": st.launches,
                     "avg_launch_ms": st.kernel_ms / max(st.launches, 1),
                     "step_kernel_share": kernel_s / t_run},
    }
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the oracle on a sample of the batch")
        out["cpu_baseline"] = cpu_baseline(args.events, args.energy, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
