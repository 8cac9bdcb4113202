"""Single-step parity: the HIP step kernel against the oracle's step on identical
states and identical Philox streams (FP64, tolerance 1e-12 relative).

Each input state (random species, energy 10 keV - 100 GeV, volume, position --
a quarter of them exactly on a boundary plane --, direction, key, step count and
interaction lengths left) is stepped once by both.  Outputs are matched by their
96-bit key: the surviving parent keeps its key, secondaries carry keys derived
from it.  Tolerances (relative error with a floor): positions 1e-12 x max(|x|,
1 cm); directions 1e-12; kinetic energies, deposits, escaped energy 1e-12 x the
input kinetic energy; step lengths 1e-12 x max(s, 1 cm); interaction lengths
1e-12 x max(|n|, 1); integers (species, volume, step count, process, limiter,
secondary counts) exactly.
"""
import numpy as np
import pytest

import workloads as W

pytestmark = pytest.mark.gpu
TOL = 1e-12


def _ctx_for(wl, n, precision=0):
    import paper_2203_09467_amd as ems
    ctx = ems.Context(pool_capacity=max(4 * n, 1024), max_events=max(n, 1), max_bins=wl.geometry.n_bins,
                      queue_capacity=1024, seed=wl.seed, precision=precision)
    ctx.setup(wl.materials, wl.options, wl.geometry)
    return ctx


def _states(wl, n, seed, species=None, e_lo=0.01, e_hi=1e5):
    g = wl.geometry
    st = W.random_track_states(n, g.n_vol, seed, e_lo=e_lo, e_hi=e_hi, species=species,
                               bounds=g.bounds, half_xy=g.half_x)
    st["event"] = np.zeros(n, np.uint32)
    return st


def _compare(wl, st, records, out, ores):
    n = len(st["species"])
    gpu = {}
    for j in range(len(out["T"])):
        gpu[(int(out["k0"][j]), int(out["k1"][j]), int(out["k2"][j]))] = j
    assert len(gpu) == len(out["T"]), "duplicate keys among GPU outputs"
    n_oracle_out = 0
    bad = []
    for i in range(n):
        r, g = ores[i], records[i]
        T_in = float(st["energy"][i])
        ok = (r.limiter == g["limiter"] and r.process == g["process"] and r.n_pair == g["n_pair"]
              and r.n_annih == g["n_annih"] and r.n_out == g["n_out"] and r.escaped == g["escaped"])
        ok &= abs(r.dep - g["dep"]) <= TOL * T_in
        ok &= abs(r.esc - g["esc"]) <= TOL * T_in
        ok &= abs(r.killed - g["killed"]) <= TOL * T_in
        ok &= abs(r.step_len - g["step_len"]) <= TOL * max(abs(r.step_len), 1.0)
        for k in range(r.n_out):
            t = r.out[k]
            n_oracle_out += 1
            j = gpu.get((t.key[0], t.key[1], t.key[2]))
            if j is None:
                ok = False
                continue
            ok &= (out["species"][j] == t.species and out["vol"][j] == t.vol and
                   out["nstep"][j] == t.nstep and out["vcap"][j] == t.vac_caps)
            for f, v in (("x", t.x), ("y", t.y), ("z", t.z)):
                ok &= abs(out[f][j] - v) <= TOL * max(abs(v), 1.0)
            for f, v in (("u", t.u), ("v", t.v), ("w", t.w)):
                ok &= abs(out[f][j] - v) <= TOL
            ok &= abs(out["T"][j] - t.T) <= TOL * T_in
            ok &= abs(out["nlam"][j] - t.nlam) <= TOL * max(abs(t.nlam), 1.0)
        if not ok:
            bad.append(i)
    assert n_oracle_out == len(out["T"])
    return bad


@pytest.mark.parametrize("n,seed", [(20000, 101), (777, 7)])
def test_calorimeter_step_parity(orc, n, seed):
    wl = W.calorimeter(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    st = _states(wl, n, seed)
    ctx = _ctx_for(wl, n)
    records, out = ctx.step_once(st)
    ores = w.step_tracks(wl.seed, st)
    bad = _compare(wl, st, records, out, ores)
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"
    # the sample exercises every limiter and every process of every species
    lim = records["limiter"]
    assert set(np.unique(lim)) == {0, 1, 2}
    for s, procs in ((0, {0, 1, 2}), (1, {0, 1}), (2, {0, 1, 2})):
        sel = (st["species"] == s) & (lim == 1)
        assert procs <= set(np.unique(records["process"][sel])) | {-1}, s


def test_low_energy_and_threshold_states(orc):
    """Energies just above the tracking cut, the pair threshold and the delta-ray threshold."""
    wl = W.calorimeter(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    n = 6000
    st = _states(wl, n, 55, e_lo=0.0101, e_hi=3.0)
    ctx = _ctx_for(wl, n)
    records, out = ctx.step_once(st)
    bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"
    assert (records["n_out"] == 0).any()  # range-outs and absorptions


def test_photon_cube_step_parity(orc):
    wl = W.photon_cube(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    n = 5000
    st = _states(wl, n, 9, species=np.zeros(n, np.int32), e_lo=0.011, e_hi=100.0)
    st["pos"][:, :2] = np.clip(st["pos"][:, :2], -5, 5)
    ctx = _ctx_for(wl, n)
    records, out = ctx.step_once(st)
    bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
    assert not bad, f"{len(bad)} of {n} states differ, first {bad[:5]}"


def test_step_once_ragged_and_single(orc):
    wl = W.calorimeter(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    for n in (1, 63, 65, 129):
        st = _states(wl, n, 1000 + n)
        ctx = _ctx_for(wl, n)
        records, out = ctx.step_once(st)
        bad = _compare(wl, st, records, out, w.step_tracks(wl.seed, st))
        assert not bad, (n, bad)
