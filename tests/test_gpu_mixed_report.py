"""Error of the mixed-precision step against the FP64 oracle, per observable.

Mixed precision runs cross-section tables, interpolation, interaction lengths and
sampling in FP32 (positions, directions, energies and tallies stay FP64).  One step
of 20 000 random calorimeter states (all species, 10 keV - 100 GeV, a quarter on
boundary planes) is taken by the mixed-precision kernel and by the oracle on the
same Philox streams, and compared per observable:
* how often the step limiter and, for interactions, the selected process agree;
* relative error of the step length (same limiter), of the parent's post-step
  kinetic energy (parent alive in both) and of the energy deposited (per input
  kinetic energy), as quantiles.
The report is printed (one JSON line) and held to bounds that a mistake in the
FP32 path -- a wrong table, a dropped term -- would break by orders of magnitude.
"""
import json

import numpy as np
import pytest

import workloads as W
from test_gpu_step_parity import _ctx_for, _states

pytestmark = pytest.mark.gpu


def test_mixed_step_error_per_observable(orc):
    wl = W.calorimeter(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    n = 20000
    st = _states(wl, n, 4242)
    ctx = _ctx_for(wl, n, precision=1)
    rec, out = ctx.step_once(st)
    ores = w.step_tracks(wl.seed, st)
    keys = {(int(out["k0"][j]), int(out["k1"][j]), int(out["k2"][j])): j for j in range(len(out["T"]))}
    lim_same = np.array([r.limiter == g["limiter"] for r, g in zip(ores, rec)])
    inter = np.array([r.limiter == 1 and g["limiter"] == 1 for r, g in zip(ores, rec)])
    proc_same = np.array([r.process == g["process"] for r, g in zip(ores, rec)])[inter]
    s_err, t_err, d_err = [], [], []
    for i, (r, g) in enumerate(zip(ores, rec)):
        T_in = float(st["energy"][i])
        if r.limiter == g["limiter"]:
            s_err.append(abs(g["step_len"] - r.step_len) / max(r.step_len, 1e-300) if r.step_len > 0
                         else abs(g["step_len"]))
        d_err.append(abs(g["dep"] - r.dep) / T_in)
        if r.parent_alive:
            t = r.out[0]
            j = keys.get((t.key[0], t.key[1], t.key[2]))
            if j is not None and t.T > 0:
                t_err.append(abs(out["T"][j] - t.T) / t.T)
    q = lambda a: {p: float(np.quantile(a, p / 100)) for p in (50, 99, 99.9)}
    report = {"states": n, "limiter_agreement": float(lim_same.mean()),
              "process_agreement": float(proc_same.mean()), "interactions_compared": int(inter.sum()),
              "step_length_rel_err": q(np.array(s_err)), "parent_T_rel_err": q(np.array(t_err)),
              "deposit_err_per_T_in": q(np.array(d_err))}
    print("MIXED_STEP_REPORT " + json.dumps(report))
    assert report["limiter_agreement"] >= 0.995
    assert report["process_agreement"] >= 0.995
    assert report["step_length_rel_err"][50] <= 1e-5
    assert report["parent_T_rel_err"][50] <= 1e-5
    assert report["deposit_err_per_T_in"][50] <= 1e-5
