"""Benchmark: electromagnetic-shower transport throughput on one MI355X.

Workload (default): 1e5 primary 1 GeV electrons at normal incidence on the
50-layer 2 mm Pb + 5 mm LAr calorimeter (40 x 40 cm), full e-/e+/photon physics,
0.7 mm production cut, FP64, seed 2.  One benchmark "step" is the transport of
the whole batch to completion (every step of the hot path: admission, cross
sections, interaction lengths, step limits, boundaries, continuous loss,
interactions, secondaries, compaction, tallies) with the primaries already
resident in HBM.  value = track-steps / s over the timed steps.

Also reported: the step kernels against the HBM roofline (algorithmic bytes =
160 B per FP64 track-step -- the minimal track state read and written by a fused
step -- times the track-steps of an iteration, divided by the step kernels'
HIP-event duration per iteration on their launch stream; the bytes this design
moves per iteration and the counter-measured traffic are reported beside it),
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
QUEUE_BYTES = 80      # queue entry: 7 doubles + 6 words (no interaction length)
# algorithmic bytes per track-step of a fused step with the minimal state (read +
# write): FP64, and mixed precision with an FP32 interaction length
BYTES_PER_STEP = {"fp64": 160, "mixed": 152}


def state_bytes(st):
    """Bytes this design moves: state read and written once per launch, queue round trips."""
    return BYTES_PER_TRACK * (st.tracks_in + st.tracks_out) + 2 * QUEUE_BYTES * st.queued


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
                       f"{wall:.1f} s wall, {len(jobs)} processes)",
                one_core_value=rate1, one_core_sample=f"events 0..19 ({steps} track-steps) in one process")


TRAFFIC_FILE = os.path.join(ROOT, "profiles", "step_kernels_calorimeter_fp64_traffic.json")


def measured_traffic(args):
    """HBM bytes per step iteration from the committed FETCH_SIZE / WRITE_SIZE counters
    of the default FP64 calorimeter workload, or None when they do not apply (another
    workload or precision, or kernel code changed since they were taken)."""
    if args.precision != "fp64" or args.events != 100_000 or args.energy != 1000.0:
        return None
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
        sha = kernel_source_digest(os.path.join(ROOT, t["kernel_source"]))
        same = (sha == t["kernel_code_sha256"] and t["energy_budget_MeV"] == args.budget and
                t["pool_slots"] == args.pool and t["iterations_per_sync"] == args.per_sync)
    except (OSError, KeyError, ValueError):
        return None
    return float(t["bytes_per_iteration"]) if same else None


def kernel_source_digest(path):
    """sha256 of a C++ source with comments and blank space removed (code only)."""
    import hashlib
    import re
    with open(path) as f:
        src = f.read()
    src = re.sub(r"//[^\n]*", "", src)
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    src = " ".join(src.split())
    return hashlib.sha256(src.encode()).hexdigest()


def run_transport(ems, wl, n_events, args, precision, log_name):
    """Transport the whole batch args.warmup + args.steps times; returns the timed totals."""
    import torch
    n_steps = args.warmup + args.steps
    ctx = ems.Context(pool_capacity=args.pool, max_events=n_events * n_steps,
                      max_bins=wl.geometry.n_bins, queue_capacity=n_events, seed=wl.seed,
                      precision=precision, energy_budget=args.budget, time_steps=True,
                      iterations_per_sync=args.per_sync)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    batches = []
    for j in range(n_steps):
        ev = wl.events.subset(np.arange(n_events))
        ev.event_ids = (np.arange(n_events) + j * n_events).astype(np.uint32)
        batches.append(ems.DeviceEvents(ev))
    torch.cuda.synchronize()
    total_steps, iters, peak = 0, 0, 0
    t0 = time.perf_counter()
    for j in range(n_steps):
        timed = j >= args.warmup
        if timed and j == args.warmup:
            ctx.step_stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        ts = time.perf_counter()
        pr = ctx.transport(batches[j], -1)
        torch.cuda.synchronize()
        log(f"{log_name} step {j} ({'timed' if timed else 'warmup'}): {pr.track_steps} track-steps "
            f"in {time.perf_counter() - ts:.3f} s, {pr.iterations} iterations, peak pool "
            f"{pr.peak_alive}, deferred {pr.deferred}")
        if timed:
            total_steps += pr.track_steps
            iters += pr.iterations
            peak = max(peak, pr.peak_alive)
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    st = ctx.step_stats()
    ids = np.concatenate([b.ids for b in batches[args.warmup:]])
    dep, led, status = ctx.read(ids)
    assert (status == 0).all()
    bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * 0.51099895 * (led[:, 3] - led[:, 4]))
    layers = dep.reshape(len(ids), -1).sum(0)
    ctx.close()
    return dict(steps=total_steps, t=t_run, iters=iters, peak=peak, stats=st, layers=layers,
                ledger_max=float(np.abs(bal / led[:, 0]).max()))


def run_serving(ems, args, precision, rate=None):
    from paper_2203_09467_amd.serve import serve
    import workloads as W
    rate = args.serve_rate if rate is None else rate
    wl = W.serving(n_events=args.serve_events, rate_hz=rate)
    ctx = ems.Context(pool_capacity=args.pool, max_events=args.serve_events,
                      max_bins=wl.geometry.n_bins, queue_capacity=wl.events.n_primaries,
                      seed=wl.seed, precision=precision, energy_budget=args.serve_budget,
                      iterations_per_sync=min(args.serve_per_sync, args.serve_iters))
    ctx.setup(wl.materials, wl.options, wl.geometry)
    res = serve(ctx, wl.events, iterations=args.serve_iters, time_limit=300.0)
    ctx.close()
    e_mean = float(wl.events.energy.sum() / wl.events.n_events)
    return {"p50_ms": res["p50"] * 1e3, "p99_ms": res["p99"] * 1e3,
            "events": wl.events.n_events, "offered_rate_hz": rate,
            "mean_event_energy_GeV": e_mean / 1000.0,
            "track_steps_per_s": res["track_steps"] / res["wall"], "wall_s": res["wall"],
            "peak_events_in_flight": res["peak_events"]}


def run_photon_sat(ems, n, args):
    """Photon-only cube with n one-photon events in one launch sequence (the small
    photon workload at sizes that fill the GPU)."""
    import torch
    import workloads as W
    wl = W.photon_cube(n)
    ctx = ems.Context(pool_capacity=4 * n, max_events=n, max_bins=wl.geometry.n_bins,
                      queue_capacity=n, seed=wl.seed, precision=ems.EMS_FP64, time_steps=True,
                      iterations_per_sync=args.per_sync)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    dev = ems.DeviceEvents(wl.events)
    torch.cuda.synchronize()
    ctx.step_stats(reset=True)
    t0 = time.perf_counter()
    pr = ctx.transport(dev, -1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = ctx.step_stats()
    ctx.close()
    kernel_s = st.kernel_ms / 1e3
    achieved = BYTES_PER_STEP["fp64"] * pr.track_steps / kernel_s / 1e9 if kernel_s > 0 else 0.0
    log(f"photon cube {n}: {pr.track_steps} track-steps in {t:.3f} s, {pr.iterations} iterations")
    return {"primaries": n, "value": pr.track_steps / t, "unit": "track-steps/s",
            "step_kernels_value": pr.track_steps / kernel_s if kernel_s > 0 else None,
            "iterations": pr.iterations, "peak_tracks_in_flight": pr.peak_alive,
            "roofline_achieved_gbs": achieved, "roofline_frac": achieved / HBM_PEAK_GBS}


def run_barrel(ems, n, args, precision):
    """Barrel with B_z = 1 T: n events of one primary (60/20/20 % e-/e+/photon,
    log-uniform 1-100 GeV, |eta| < 1.5), RK4 field propagation."""
    import torch
    import workloads as W
    wl = W.barrel(n)
    ctx = ems.Context(pool_capacity=args.pool, max_events=n, max_bins=wl.geometry.n_bins,
                      queue_capacity=n, seed=wl.seed, precision=precision, energy_budget=args.budget,
                      time_steps=True, iterations_per_sync=args.per_sync)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    dev = ems.DeviceEvents(wl.events)
    torch.cuda.synchronize()
    ctx.step_stats(reset=True)
    t0 = time.perf_counter()
    pr = ctx.transport(dev, -1)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    st = ctx.step_stats()
    dep, led, status = ctx.read(wl.events.event_ids)
    ctx.close()
    assert (status == 0).all()
    bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * 0.51099895 * (led[:, 3] - led[:, 4]))
    kernel_s = st.kernel_ms / 1e3
    per_step = BYTES_PER_STEP["fp64" if precision == ems.EMS_FP64 else "mixed"]
    achieved = per_step * pr.track_steps / kernel_s / 1e9 if kernel_s > 0 else 0.0
    log(f"barrel {n} ({'fp64' if precision == ems.EMS_FP64 else 'mixed'}): {pr.track_steps} "
        f"track-steps in {t:.3f} s, {pr.iterations} iterations")
    return {"value": pr.track_steps / t, "unit": "track-steps/s", "track_steps": pr.track_steps,
            "iterations": pr.iterations, "peak_tracks_in_flight": pr.peak_alive,
            "roofline_achieved_gbs": achieved, "roofline_frac": achieved / HBM_PEAK_GBS,
            "ledger_max_rel_error": float(np.abs(bal / led[:, 0]).max())}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--events", type=int, default=100_000)
    ap.add_argument("--energy", type=float, default=1000.0, help="primary energy, MeV")
    ap.add_argument("--precision", choices=["fp64", "mixed"], default="fp64")
    ap.add_argument("--pool", type=int, default=1 << 24)
    ap.add_argument("--budget", type=float, default=1e8, help="energy in flight, MeV")
    ap.add_argument("--per-sync", type=int, default=4,
                    help="step iterations launched back to back between host synchronisations")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-mixed", action="store_true", help="skip the mixed-precision leg")
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-barrel", action="store_true", help="skip the barrel (field) runs")
    ap.add_argument("--barrel-events", type=int, default=20_000)
    ap.add_argument("--no-photon-sat", action="store_true",
                    help="skip the photon-cube runs at 1e6 and 1e7 primaries")
    ap.add_argument("--serve-events", type=int, default=1000)
    ap.add_argument("--serve-budget", type=float, default=5e7,
                    help="energy in flight of the serving loop, MeV")
    ap.add_argument("--serve-rate", type=float, default=40.0, help="offered events/s")
    ap.add_argument("--serve-rate-high", type=float, default=120.0,
                    help="a second, higher offered load (events/s); 0 skips it")
    ap.add_argument("--serve-per-sync", type=int, default=4,
                    help="iterations per host synchronisation in the serving loop")
    ap.add_argument("--serve-iters", type=int, default=32,
                    help="step iterations per transport call of the serving loop")
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

    import paper_2203_09467_amd as ems
    import workloads as W

    seed = 2
    wl = W.calorimeter(args.events, energy=args.energy, seed=seed)
    prec = ems.EMS_FP64 if args.precision == "fp64" else ems.EMS_MIXED
    r = run_transport(ems, wl, args.events, args, prec, args.precision)
    value = r["steps"] / r["t"]
    st = r["stats"]
    kernel_s = st.kernel_ms / 1e3
    iters = max(st.launches, 1)
    # algorithmic bytes of one launch (iteration): the per-track-step figure times the
    # track-steps the launch performs
    bytes_alg = BYTES_PER_STEP[args.precision] * r["steps"] / iters
    achieved = bytes_alg / (kernel_s / iters) / 1e9 if kernel_s > 0 else 0.0
    traffic = measured_traffic(args)
    out = {
        "metric": "track-steps/s (FP64 vs mixed-prec) + p50/p99 event latency, 1 MI355X",
        "value": value,
        "unit": "track-steps/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": r["t"] / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if prec == ems.EMS_FP64 else "f32+f64",
        "data": "synthetic",
        "config": {"workload": f"calorimeter: {args.events} x {args.energy / 1000:g} GeV e- on "
                               "50 x (2 mm Pb + 5 mm LAr), 40x40 cm, 0.7 mm cut, seed 2",
                   "precision": args.precision, "pool_slots": args.pool,
                   "energy_budget_MeV": args.budget, "iterations_per_sync": args.per_sync,
                   "iterations": r["iters"],
                   "peak_tracks_in_flight": r["peak"], "track_steps": r["steps"],
                   "ledger_max_rel_error": r["ledger_max"]},
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
                     "traffic_unit": "bytes per iteration",
                     "measured_gbs": None if traffic is None else traffic / (kernel_s / iters) / 1e9,
                     "algorithmic_bytes_per_iteration": bytes_alg,
                     "algorithmic_bytes_per_track_step": BYTES_PER_STEP[args.precision],
                     "track_steps_per_iteration": r["steps"] / iters,
                     "state_bytes_per_iteration": state_bytes(st) / iters,
                     "kernel": "step kernels (k_transport + k_interact)",
                     "launches": st.launches,
                     "avg_iteration_ms": st.kernel_ms / max(st.launches, 1),
                     "step_kernel_share": kernel_s / r["t"]},
    }
    if args.precision == "fp64" and not args.no_mixed:
        m = run_transport(ems, wl, args.events, args, ems.EMS_MIXED, "mixed")
        big = r["layers"] >= 0.01 * r["layers"].sum()
        rel = np.abs(m["layers"] - r["layers"])[big] / r["layers"][big]
        out["mixed"] = {"value": m["steps"] / m["t"], "unit": "track-steps/s",
                        "speedup_vs_fp64": (m["steps"] / m["t"]) / value,
                        "max_rel_dev_per_bin_vs_fp64": float(rel.max()),
                        "ledger_max_rel_error": m["ledger_max"]}
    if not args.no_serving:
        log("serving: Poisson arrivals, FP64 then mixed")
        out["serving"] = {"fp64": run_serving(ems, args, ems.EMS_FP64),
                          "mixed": run_serving(ems, args, ems.EMS_MIXED),
                          "workload": "calorimeter geometry; events of U{1..500} primaries "
                                      "(60/20/20% e-/e+/photon), log-uniform 1-100 GeV, seed 5"}
        if args.serve_rate_high > 0:
            r2 = args.serve_rate_high
            out["serving"]["higher_load"] = {"offered_rate_hz": r2,
                                             "fp64": run_serving(ems, args, ems.EMS_FP64, r2),
                                             "mixed": run_serving(ems, args, ems.EMS_MIXED, r2)}
    if not args.no_barrel:
        fm = run_barrel(ems, args.barrel_events, args, ems.EMS_MIXED)
        fd = run_barrel(ems, args.barrel_events, args, ems.EMS_FP64)
        out["barrel_field"] = {
            "workload": f"{args.barrel_events} primaries (60/20/20 % e-/e+/photon), log-uniform "
                        "1-100 GeV, |eta| < 1.5, barrel of 5 Si shells + 50 Pb/LAr layers, "
                        "B_z = 1 T, RK4 tolerance 1e-5 cm, seed 4",
            "mixed": fm, "fp64": fd, "mixed_speedup_vs_fp64": fm["value"] / fd["value"]}
    if not args.no_photon_sat:
        out["photon_cube_sat"] = {
            "workload": "10 MeV photons into a 10 cm Pb cube, one photon per event, FP64",
            "runs": [run_photon_sat(ems, n, args) for n in (1_000_000, 10_000_000)]}
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the oracle on a sample of the batch")
        out["cpu_baseline"] = cpu_baseline(args.events, args.energy, seed)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
