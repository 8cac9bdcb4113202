"""Benchmark: electromagnetic-shower transport throughput on one MI355X.

Headline workload: 1e6 primary 10 GeV electrons at normal incidence on the
50-layer 2 mm Pb + 5 mm LAr calorimeter (40 x 40 cm), full e-/e+/photon physics,
0.7 mm production cut, seed 3, transported in FP64 and then in mixed precision
on identical random streams.  The primaries of the whole batch are resident in
HBM before timing starts.  The timed steps together cover every one of the 1e6
events: step j transports slice j of the batch to completion (every part of the
hot path: admission, cross sections, interaction lengths, step limits,
boundaries, continuous loss, interactions, secondaries, compaction, tallies)
and reads its tallies back, which releases the slice's event slots for the next
one.  Warmup steps transport slices of other event ids.  value = FP64
track-steps / s over the timed steps; the mixed-precision rate, its per-layer
deviation from FP64 and its speed-up are reported beside it.

Also reported: the step kernels against the HBM roofline (algorithmic bytes =
160 B per FP64 track-step -- the minimal track state read and written by a fused
step -- times the track-steps of an iteration, divided by the step kernels'
HIP-event duration per iteration on their launch stream; the bytes this design
moves per iteration and the counter-measured traffic are reported beside it),
and the CPU oracle timed on a bounded sample of the same events on the host
cores (cpu_baseline), whose per-event tallies are compared with the GPU's.
"""
import argparse
import glob
import json
import math
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
ME = 0.51099895
BYTES_PER_TRACK = 88  # SoA state of one track: 8 doubles + 6 words
QUEUE_BYTES = 80      # queue entry: 7 doubles + 6 words (no interaction length)
# algorithmic bytes per track-step of a fused step with the minimal state (read +
# write): FP64, and mixed precision with an FP32 interaction length
BYTES_PER_STEP = {"fp64": 160, "mixed": 152}
# the machine's CPU share for one GPU
CPU_SHARE = 16


def state_bytes(st):
    """Bytes this design moves: state read and written once per launch, queue round trips."""
    return BYTES_PER_TRACK * (st.tracks_in + st.tracks_out) + 2 * QUEUE_BYTES * st.queued


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_description():
    try:
        cores = len(os.sched_getaffinity(0))
    except AttributeError:
        cores = os.cpu_count() or 1
    model = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpus_visible": cores, "cpu_model": model, "logical_cpus_total": os.cpu_count()}


def _oracle_worker(args):
    seed, lo, hi, n_events, energy = args
    import oracle
    import workloads as W
    wl = W.calorimeter(hi - lo, energy=energy, seed=seed, first_id=lo)  # events lo .. hi-1
    w = oracle.World(wl.materials, wl.options, wl.geometry)
    ev = wl.events
    t0 = time.perf_counter()
    r = w.run_events(wl.seed, ev)
    return int(r["steps"].sum()), time.perf_counter() - t0, r["dep"], r["ledger"]


def cpu_baseline(n_events, energy, seed, budget_s=15.0):
    """The oracle as it stands, events split across processes on the host cores;
    returns the rate and the per-event tallies of the sample."""
    import multiprocessing as mp
    host = host_description()
    workers = max(1, min(host["cpus_visible"], CPU_SHARE))
    # calibrate on a few events, then size the sample for ~budget_s of wall time
    steps, dt, _, _ = _oracle_worker((seed, 0, 4, n_events, energy))
    rate1 = steps / max(dt, 1e-9)
    per_event = steps / 4
    n_sample = int(min(n_events, max(workers * 4, rate1 * budget_s * workers / per_event)))
    chunks = np.linspace(0, n_sample, workers + 1).astype(int)
    jobs = [(seed, int(a), int(b), n_events, energy) for a, b in zip(chunks[:-1], chunks[1:]) if b > a]
    t0 = time.perf_counter()
    with mp.get_context("spawn").Pool(len(jobs)) as pool:
        res = pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    total = sum(r[0] for r in res)
    dep = np.concatenate([r[2] for r in res])
    led = np.concatenate([r[3] for r in res])
    out = dict(value=total / wall, unit="track-steps/s", cores=len(jobs), kind="oracle",
               sample=f"events 0..{n_sample - 1} of the benchmark batch ({total} track-steps, "
                      f"{wall:.1f} s wall, {len(jobs)} processes, one per core)",
               one_core_value=rate1, one_core_sample=f"events 0..3 ({steps} track-steps) in one process",
               host=host, note=f"worker count = min(visible CPUs, {CPU_SHARE}), the box's CPU share "
                               "for one GPU")
    return out, dep, led


def _batch_sigma(x, n_batches=20):
    n = x.shape[0] // n_batches * n_batches
    b = x[:n].reshape(n_batches, -1, x.shape[1]).mean(1)
    return b.std(0, ddof=1) / math.sqrt(n_batches)


def compare_layers(g, o, rel_bar):
    """Per layer (Pb + LAr of each of the 50 layers): |mean_G - mean_O| against
    3 sigma (batch means of both) + rel_bar |mean_O|; returns the worst ratio."""
    lg = g.reshape(g.shape[0], -1, 2).sum(2)
    lo = o.reshape(o.shape[0], -1, 2).sum(2)
    sg, so = _batch_sigma(lg), _batch_sigma(lo)
    mg, mo = lg.mean(0), lo.mean(0)
    allowed = 3 * np.sqrt(sg ** 2 + so ** 2) + rel_bar * np.abs(mo) + 1e-300
    ratio = np.abs(mg - mo) / allowed
    return float(ratio.max()), bool((ratio <= 1.0).all())


TRAFFIC_GLOB = os.path.join(ROOT, "profiles", "*_traffic.json")


def measured_traffic(args, precision=None):
    """HBM bytes per step iteration from a committed FETCH_SIZE / WRITE_SIZE profile
    taken with the same workload, precision and run settings, or None when none
    applies (kernel code changed since, or other settings)."""
    precision = precision or args.precision
    for path in sorted(glob.glob(TRAFFIC_GLOB)):
        try:
            with open(path) as f:
                t = json.load(f)
            sha = kernel_source_digest(os.path.join(ROOT, t["kernel_source"]))
            # the counters are taken on a sample of the batch with the same per-event
            # energy, in-flight budget, pool and sync interval: the pool holds the same
            # mix of showers, so the bytes per iteration carry over
            same = (sha == t["kernel_code_sha256"] and t["precision"] == precision and
                    t["energy_MeV"] == args.energy and
                    t["energy_budget_MeV"] == args.budget and t["pool_slots"] == args.pool and
                    t["iterations_per_sync"] == args.per_sync)
        except (OSError, KeyError, ValueError):
            continue
        if same:
            return float(t["bytes_per_iteration"])
    return None


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


def run_transport(ems, args, precision, log_name, keep):
    """Transport the batch in args.steps timed slices after args.warmup slices of other
    event ids; each slice runs to completion and its tallies are read (slots released)
    inside the timed region.  Returns the timed totals, the per-layer sums over the
    whole batch and the per-event tallies of events 0..keep-1."""
    import torch
    import workloads as W
    n = args.events
    per = -(-n // args.steps)
    n_all = n + args.warmup * per
    wl = W.calorimeter(n_all, energy=args.energy, seed=args.seed)
    ctx = ems.Context(pool_capacity=args.pool, max_events=per, max_bins=wl.geometry.n_bins,
                      queue_capacity=per, seed=wl.seed, precision=precision,
                      energy_budget=args.budget, time_steps=True, iterations_per_sync=args.per_sync)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    dev = ems.DeviceEvents(wl.events)  # every primary of every slice resident in HBM
    # warmup slices: ids n .. n_all-1; timed slices: ids 0 .. n-1
    slices = [(n + j * per, n + (j + 1) * per) for j in range(args.warmup)]
    slices += [(j * per, min(n, (j + 1) * per)) for j in range(args.steps)]
    layers = np.zeros(wl.geometry.n_bins)
    kept_dep, kept_led = [], []
    shape = None
    ledger_max = 0.0
    total_steps, iters, peak, step_s = 0, 0, 0, []
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for j, (a, b) in enumerate(slices):
        timed = j >= args.warmup
        if timed and j == args.warmup:
            ctx.step_stats(reset=True)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
        ts = time.perf_counter()
        pr = ctx.transport(dev.slice(a, b), -1)
        dep, led, status = ctx.read(wl.events.event_ids[a:b])
        dt = time.perf_counter() - ts
        if j == args.warmup:  # the first timed slice: per-iteration shape of one transport
            shape = characterise(ctx.iteration_log(reset=True))
        else:
            ctx.iteration_log(reset=True)
        assert (status == 0).all() and pr.alive == 0
        log(f"{log_name} step {j} ({'timed' if timed else 'warmup'}): events {a}..{b - 1}, "
            f"{pr.track_steps} track-steps in {dt:.3f} s, {pr.iterations} iterations, peak pool "
            f"{pr.peak_alive}, deferred {pr.deferred}")
        if timed:
            total_steps += pr.track_steps
            iters += pr.iterations
            peak = max(peak, pr.peak_alive)
            step_s.append(dt)
            layers += dep.sum(0)
            bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * ME * (led[:, 3] - led[:, 4]))
            ledger_max = max(ledger_max, float(np.abs(bal / led[:, 0]).max()))
            if a < keep:
                m = min(b, keep) - a
                kept_dep.append(dep[:m].copy())
                kept_led.append(led[:m].copy())
    torch.cuda.synchronize()
    t_run = time.perf_counter() - t0
    st = ctx.step_stats()
    ctx.close()
    return dict(steps=total_steps, t=t_run, iters=iters, peak=peak, stats=st, layers=layers,
                ledger_max=ledger_max, step_s=step_s, per=per, shape=shape,
                kept_dep=np.concatenate(kept_dep) if kept_dep else None,
                kept_led=np.concatenate(kept_led) if kept_led else None)


def characterise(log):
    """The per-iteration shape of one transport (the paper's characterisation of the
    GPU loop): iterations to reach 90 % of the peak pool, share of iterations after
    the peak with the pool below half of it (draining), shortest over longest
    iteration time."""
    if len(log) == 0:
        return None
    n = log["photons"].astype(np.int64) + log["charged"]
    peak = int(n.max())
    k_peak = int(np.argmax(n))
    rise = int(np.argmax(n >= 0.9 * peak)) + 1
    drain = int((n[k_peak:] < 0.5 * peak).sum())
    ms = log["ms"]
    return {"iterations": int(len(log)), "peak_tracks": peak, "iterations_to_90pct_of_peak": rise,
            "draining_share": drain / len(log),
            "min_over_max_iteration_time": float(ms.min() / ms.max()) if ms.max() > 0 else None,
            "interactions_per_iteration_at_peak": int(log["interactions"][k_peak])}


def run_serving_batch(ems, args, precision):
    """The serving workload's events submitted at once and run to completion (the
    batch rate of the same events, against which the serving loop saturates)."""
    import torch
    import workloads as W
    wl = W.serving(n_events=args.serve_events, rate_hz=args.serve_rate)
    ctx = ems.Context(pool_capacity=args.pool, max_events=args.serve_events,
                      max_bins=wl.geometry.n_bins, queue_capacity=wl.events.n_primaries,
                      seed=wl.seed, precision=precision, energy_budget=args.serve_budget,
                      iterations_per_sync=args.serve_per_sync, spill_capacity=args.serve_spill)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    dev = ems.DeviceEvents(wl.events)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    pr = ctx.transport(dev, -1)
    dep, led, status = ctx.read(wl.events.event_ids)
    torch.cuda.synchronize()
    t = time.perf_counter() - t0
    ctx.close()
    assert (status == 0).all()
    return {"track_steps_per_s": pr.track_steps / t, "wall_s": t, "iterations": pr.iterations,
            "peak_tracks_in_flight": pr.peak_alive}


def run_serving(ems, args, precision, rate=None):
    from paper_2203_09467_amd.serve import serve
    import workloads as W
    rate = args.serve_rate if rate is None else rate
    wl = W.serving(n_events=args.serve_events, rate_hz=rate)
    ctx = ems.Context(pool_capacity=args.pool, max_events=args.serve_events,
                      max_bins=wl.geometry.n_bins, queue_capacity=wl.events.n_primaries,
                      seed=wl.seed, precision=precision, energy_budget=args.serve_budget,
                      iterations_per_sync=min(args.serve_per_sync, args.serve_iters),
                      spill_capacity=args.serve_spill)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    res = serve(ctx, wl.events, iterations=args.serve_iters, time_limit=300.0)
    ctx.close()
    e_mean = float(wl.events.energy.sum() / wl.events.n_events)
    return {"p50_ms": res["p50"] * 1e3, "p99_ms": res["p99"] * 1e3,
            "events": wl.events.n_events, "offered_rate_hz": rate,
            "mean_event_energy_GeV": e_mean / 1000.0,
            "track_steps_per_s": res["track_steps"] / res["wall"], "wall_s": res["wall"],
            "peak_events_in_flight": res["peak_events"]}


def run_csg(ems, n, args, precision):
    """The quadric-cell module (spheres, an x-cylinder, a cone, planes): n events of one
    primary from its centre; and the calorimeter written as cells next to its slab
    navigation (same results bitwise), for the cost of general navigation."""
    import torch
    import workloads as W
    out = {}
    for name, wl in (("module", W.csg_module(n)),
                     ("calorimeter_as_cells", W.Workload("c", W.calorimeter(1).materials,
                                                         W.calorimeter(1).options,
                                                         W.calorimeter_csg(),
                                                         W.calorimeter(n // 10).events, 2)),
                     ("calorimeter_slabs", W.calorimeter(n // 10))):
        ne = wl.events.n_events
        ctx = ems.Context(pool_capacity=args.pool, max_events=ne, max_bins=wl.geometry.n_bins,
                          queue_capacity=wl.events.n_primaries, seed=wl.seed, precision=precision,
                          energy_budget=args.budget, time_steps=True, iterations_per_sync=args.per_sync)
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
        bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * ME * (led[:, 3] - led[:, 4]))
        log(f"quadric cells {name} {ne}: {pr.track_steps} track-steps in {t:.3f} s")
        out[name] = {"events": ne, "value": pr.track_steps / t, "unit": "track-steps/s",
                     "step_kernels_value": pr.track_steps / (st.kernel_ms / 1e3),
                     "track_steps": pr.track_steps,
                     "ledger_max_rel_error": float(np.abs(bal / led[:, 0]).max())}
    out["workload"] = ("module: 40 cm Pb cube, Si spherical shell 8-10 cm, LAr, W rod r = 3 cm "
                       "along x, conical vacuum channel; one primary per event from the centre, "
                       "60/20/20 % e-/e+/photon, log-uniform 0.1-10 GeV, seed 7; calorimeter "
                       f"1 GeV e-, {n // 10} events, as quadric cells and as slabs")
    return out


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
    bal = led[:, 0] - (dep.sum(1) + led[:, 1] + led[:, 2] + 2 * ME * (led[:, 3] - led[:, 4]))
    kernel_s = st.kernel_ms / 1e3
    per_step = BYTES_PER_STEP["fp64" if precision == ems.EMS_FP64 else "mixed"]
    achieved = per_step * pr.track_steps / kernel_s / 1e9 if kernel_s > 0 else 0.0
    log(f"barrel {n} ({'fp64' if precision == ems.EMS_FP64 else 'mixed'}): {pr.track_steps} "
        f"track-steps in {t:.3f} s, {pr.iterations} iterations")
    return {"value": pr.track_steps / t, "unit": "track-steps/s", "track_steps": pr.track_steps,
            "iterations": pr.iterations, "peak_tracks_in_flight": pr.peak_alive,
            "roofline_achieved_gbs": achieved, "roofline_frac": achieved / HBM_PEAK_GBS,
            "ledger_max_rel_error": float(np.abs(bal / led[:, 0]).max())}


def roofline(r, precision, traffic):
    st = r["stats"]
    kernel_s = st.kernel_ms / 1e3
    iters = max(st.launches, 1)
    # algorithmic bytes of one launch (iteration): the per-track-step figure times the
    # track-steps the launch performs
    bytes_alg = BYTES_PER_STEP[precision] * r["steps"] / iters
    iter_s = kernel_s / iters
    achieved = bytes_alg / iter_s / 1e9 if kernel_s > 0 else 0.0
    return {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
            "frac": achieved / HBM_PEAK_GBS, "traffic": traffic,
            "traffic_unit": "HBM bytes per iteration (FETCH_SIZE + WRITE_SIZE, scaled)",
            "measured_gbs": None if traffic is None else traffic / iter_s / 1e9,
            "measured_frac": None if traffic is None else traffic / iter_s / 1e9 / HBM_PEAK_GBS,
            "algorithmic_bytes_per_iteration": bytes_alg,
            "algorithmic_bytes_per_track_step": BYTES_PER_STEP[precision],
            "track_steps_per_iteration": r["steps"] / iters,
            "state_bytes_per_iteration": state_bytes(st) / iters,
            "kernel": "step kernels (k_transport + k_interact), one iteration per launch pair",
            "launches": st.launches, "avg_iteration_ms": st.kernel_ms / iters,
            "step_kernel_share": kernel_s / r["t"]}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10,
                    help="timed steps; together they cover every event of the batch")
    ap.add_argument("--warmup", type=int, default=2, help="untimed slices of other event ids")
    ap.add_argument("--events", type=int, default=1_000_000)
    ap.add_argument("--energy", type=float, default=10_000.0, help="primary energy, MeV")
    ap.add_argument("--seed", type=int, default=3)
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
    ap.add_argument("--serve-budget", type=float, default=1e8,
                    help="kinetic energy of the pool (measured on the device) up to which the "
                         "serving loop admits events, MeV, besides free pool slots (0: slots only)")
    ap.add_argument("--serve-spill", type=int, default=1 << 23,
                    help="tracks the serving context may spill to pinned host memory")
    ap.add_argument("--serve-rate", type=float, default=40.0, help="offered events/s")
    ap.add_argument("--serve-rates-high", type=str, default="120,200,400",
                    help="higher offered loads (events/s, comma separated); empty skips them")
    ap.add_argument("--no-csg", action="store_true", help="skip the quadric-cell geometry runs")
    ap.add_argument("--csg-events", type=int, default=20_000)
    ap.add_argument("--serve-per-sync", type=int, default=4,
                    help="iterations per host synchronisation in the serving loop")
    ap.add_argument("--serve-iters", type=int, default=32,
                    help="step iterations per transport call of the serving loop")
    ap.add_argument("--barrel-only", choices=["fp64", "mixed"], default=None,
                    help="only run the barrel (field) workload of --barrel-events primaries in "
                         "this precision (for profiling the curved-move kernel)")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run a plain device copy of MIB MiB (read + write) three times, "
                         "to scale HBM byte counters")
    args = ap.parse_args()
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU; --gpus must be 1 (the path would "
                                   "shard by event, one context per GPU)"}))
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

    if args.barrel_only:
        p = ems.EMS_FP64 if args.barrel_only == "fp64" else ems.EMS_MIXED
        print(json.dumps({"barrel_field": run_barrel(ems, args.barrel_events, args, p)}))
        return
    prec = ems.EMS_FP64 if args.precision == "fp64" else ems.EMS_MIXED
    cpu = None
    keep = 0
    if not args.no_cpu_baseline:
        log("cpu baseline: timing the oracle on a sample of the batch")
        cpu, o_dep, o_led = cpu_baseline(args.events, args.energy, args.seed)
        keep = o_dep.shape[0]
    r = run_transport(ems, args, prec, args.precision, keep)
    value = r["steps"] / r["t"]
    workload = (f"calorimeter: {args.events} x {args.energy / 1000:g} GeV e- on 50 x (2 mm Pb + "
                f"5 mm LAr), 40x40 cm, 0.7 mm cut, seed {args.seed}")
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
        "config": {"workload": workload, "precision": args.precision,
                   "events_per_step": r["per"], "pool_slots": args.pool,
                   "energy_budget_MeV": args.budget, "iterations_per_sync": args.per_sync,
                   "iterations": r["iters"], "peak_tracks_in_flight": r["peak"],
                   "track_steps": r["steps"], "ledger_max_rel_error": r["ledger_max"],
                   "step_ms": [round(x * 1e3, 2) for x in r["step_s"]],
                   "step_ms_max_over_min": max(r["step_s"]) / min(r["step_s"]),
                   "characterisation_of_one_step": r["shape"]},
        "roofline": roofline(r, args.precision, measured_traffic(args)),
    }
    if cpu is not None:
        n = min(keep, r["kept_dep"].shape[0])
        g, o = r["kept_dep"][:n], o_dep[:n]
        e_in = o_led[:n, 0]
        match = np.abs(g - o).max(1) <= 1e-9 * e_in
        worst, ok = compare_layers(g, o, 1e-3 if prec == ems.EMS_FP64 else 5e-3)
        cpu["parity_vs_gpu"] = {
            "events": n, "precision": args.precision,
            "events_equal_to_1e-9_E_in": float(match.mean()),
            "per_layer_worst_ratio_to_bar": worst, "per_layer_within_bar": ok,
            "bar": "3 sigma (batch means) + 0.1 % per layer" if prec == ems.EMS_FP64 else
                   "3 sigma (batch means) + 0.5 % per layer"}
    if args.precision == "fp64" and not args.no_mixed:
        m = run_transport(ems, args, ems.EMS_MIXED, "mixed", keep)
        big = r["layers"] >= 0.01 * r["layers"].sum()
        rel = np.abs(m["layers"] - r["layers"])[big] / r["layers"][big]
        lf = r["layers"].reshape(-1, 2).sum(1)
        lm = m["layers"].reshape(-1, 2).sum(1)
        bigl = lf >= 0.01 * lf.sum()
        rel_l = np.abs(lm - lf)[bigl] / lf[bigl]
        out["mixed"] = {"value": m["steps"] / m["t"], "unit": "track-steps/s",
                        "speedup_vs_fp64": (m["steps"] / m["t"]) / value,
                        "ms_per_step": m["t"] / args.steps * 1e3,
                        "max_rel_dev_per_layer_vs_fp64": float(rel_l.max()),
                        "max_rel_dev_per_bin_vs_fp64": float(rel.max()),
                        "layers_compared": int(bigl.sum()),
                        "note": "paired on identical Philox streams over every event of the batch; "
                                "layers (Pb + LAr) and bins holding >= 1 % of the deposit",
                        "ledger_max_rel_error": m["ledger_max"],
                        "step_ms_max_over_min": max(m["step_s"]) / min(m["step_s"]),
                        "roofline": roofline(m, "mixed", measured_traffic(args, "mixed"))}
        if cpu is not None:
            n = min(keep, m["kept_dep"].shape[0])
            worst, ok = compare_layers(m["kept_dep"][:n], o_dep[:n], 5e-3)
            out["mixed"]["vs_oracle"] = {"events": n, "per_layer_worst_ratio_to_bar": worst,
                                         "per_layer_within_bar": ok,
                                         "bar": "3 sigma (batch means) + 0.5 % per layer"}
    if not args.no_serving:
        log("serving: Poisson arrivals, FP64 then mixed")
        out["serving"] = {"fp64": run_serving(ems, args, ems.EMS_FP64),
                          "mixed": run_serving(ems, args, ems.EMS_MIXED),
                          "workload": "calorimeter geometry; events of U{1..500} primaries "
                                      "(60/20/20% e-/e+/photon), log-uniform 1-100 GeV, seed 5"}
        out["serving"]["admission"] = ("by free pool slots (a quarter of the pool for new "
                                       "primaries) while the pool's kinetic energy, measured on "
                                       f"the device, stays within {args.serve_budget:g} MeV "
                                       "(0 = slots only); a pool above 3/4 full spills its "
                                       "highest-energy tracks to host memory "
                                       f"(room for {args.serve_spill} tracks)")
        out["serving"]["same_events_as_one_batch"] = {
            "fp64": run_serving_batch(ems, args, ems.EMS_FP64),
            "note": "the 1000 events submitted at once and run to completion, same admission"}
        highs = [float(x) for x in args.serve_rates_high.split(",") if x.strip()]
        out["serving"]["higher_loads"] = [
            {"offered_rate_hz": r2, "fp64": run_serving(ems, args, ems.EMS_FP64, r2),
             "mixed": run_serving(ems, args, ems.EMS_MIXED, r2)} for r2 in highs]
    if not args.no_barrel:
        fm = run_barrel(ems, args.barrel_events, args, ems.EMS_MIXED)
        fd = run_barrel(ems, args.barrel_events, args, ems.EMS_FP64)
        out["barrel_field"] = {
            "workload": f"{args.barrel_events} primaries (60/20/20 % e-/e+/photon), log-uniform "
                        "1-100 GeV, |eta| < 1.5, barrel of 5 Si shells + 50 Pb/LAr layers, "
                        "B_z = 1 T, RK4 tolerance 1e-5 cm, seed 4",
            "mixed": fm, "fp64": fd, "mixed_speedup_vs_fp64": fm["value"] / fd["value"]}
    if not args.no_csg:
        out["quadric_cells"] = run_csg(ems, args.csg_events, args, prec)
    if not args.no_photon_sat:
        out["photon_cube_sat"] = {
            "workload": "10 MeV photons into a 10 cm Pb cube, one photon per event, FP64",
            "runs": [run_photon_sat(ems, n, args) for n in (1_000_000, 10_000_000)]}
    if cpu is not None:
        out["cpu_baseline"] = cpu
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
