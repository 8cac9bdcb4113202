"""Pins of the oracle's multiple-scattering deflection (CPU only).

The paper lists multiple scattering (Urban, WentzelVI) only as in progress and
defines no model; the reading here is Highland's Gaussian width of the projected
angle, theta0 = 13.6 MeV / (beta c p) sqrt(x/X0) [1 + 0.038 ln(x / (X0 beta^2))]
(Highland 1975; Lynch and Dahl 1991), with the space angle theta0 sqrt(-2 ln u)
and a uniform azimuth.  Pinned here:
* the width at one radiation length is 13.6 MeV / (beta c p) (the log term vanishes),
  it scales as 1/(beta p), and it is zero where the bracket is not positive;
* sampled deflections: theta^2 / (2 theta0^2) is exponential with mean 1 and the
  azimuth is uniform (chi-square), from the oracle's own steps;
* with the option off nothing deflects; with it on events still conserve energy.
"""
import math

import numpy as np
from scipy import stats

import workloads as W

ME = 0.51099895


def test_width_at_one_radiation_length(orc):
    L = orc.lib()
    for T in (1.0, 30.0, 1000.0, 1e5):
        p = math.sqrt(T * (T + 2 * ME))
        beta = p / (T + ME)
        X0 = 0.56
        # at x = X0 beta^2 the logarithm is zero: theta0 = 13.6 / (beta p) * beta
        th = L.or_msc_theta0(T, X0 * beta * beta, X0)
        assert abs(th - 13.6 / (beta * p) * beta) <= 1e-14 * th
    # ultra-relativistic, x = X0: 13.6 MeV / p to the accuracy of beta = 1
    T = 1e5
    p = math.sqrt(T * (T + 2 * ME))
    assert abs(L.or_msc_theta0(T, 1.0, 1.0) * p / 13.6 - 1.0) < 1e-9
    # far below the fit's range the bracket turns negative: no deflection
    assert L.or_msc_theta0(1000.0, 1e-14, 1.0) == 0.0
    assert L.or_msc_theta0(1000.0, 0.0, 1.0) == 0.0


def _scatter_steps(orc, n, T, seed):
    wl = W.calorimeter(1)
    opts = W.Options(production_cut=0.07, msc=1, compton=0, photoelectric=0, pair=0,
                     ionisation=0, brems=0, annihilation=0)
    # one thick lead slab: steps end on the continuous-loss limit, inside the slab
    geom = W.Geometry(0, np.array([-50.0, 50.0]), np.array([0], np.int32), np.array([0], np.int32),
                      1, half_x=50.0, half_y=50.0)
    w = orc.World(wl.materials, opts, geom)
    rng = np.random.default_rng(seed)
    st = dict(species=np.full(n, W.ELECTRON, np.int32), energy=np.full(n, T), vol=np.zeros(n, np.int32),
              pos=np.zeros((n, 3)), dir=np.tile([0.0, 0.0, 1.0], (n, 1)), nlam=np.full(n, 1.0),
              key=rng.integers(0, 2 ** 32, size=(n, 3), dtype=np.uint64).astype(np.uint32),
              nstep=rng.integers(0, 1000, n).astype(np.uint32), event=np.zeros(n, np.uint32))
    res = w.step_tracks(wl.seed, st)
    X0 = w.X0(0)
    th, ph, th0 = [], [], []
    for r in res:
        assert r.parent_alive and r.limiter == 2
        d = r.out[0]
        th.append(math.acos(max(-1.0, min(1.0, d.w))))
        ph.append(math.atan2(d.v, d.u) % (2 * math.pi))
        th0.append(orc.lib().or_msc_theta0(T, r.step_len, X0))
    return np.array(th), np.array(ph), np.array(th0)


def test_sampled_deflections_follow_the_width(orc):
    th, ph, th0 = _scatter_steps(orc, 20000, 50.0, 1)
    x = th ** 2 / (2 * th0 ** 2)
    edges = stats.expon.ppf(np.linspace(0, 1, 21))
    obs, _ = np.histogram(x, edges)
    assert stats.chisquare(obs).pvalue > 1e-3
    obs, _ = np.histogram(ph, np.linspace(0, 2 * np.pi, 21))
    assert stats.chisquare(obs).pvalue > 1e-3
    assert abs(x.mean() - 1.0) < 0.03


def test_no_deflection_without_the_option(orc):
    wl = W.calorimeter(1)
    opts = W.Options(production_cut=0.07, compton=0, photoelectric=0, pair=0, ionisation=0, brems=0,
                     annihilation=0)
    geom = W.Geometry(0, np.array([-50.0, 50.0]), np.array([0], np.int32), np.array([0], np.int32),
                      1, half_x=50.0, half_y=50.0)
    w = orc.World(wl.materials, opts, geom)
    n = 200
    st = dict(species=np.full(n, W.ELECTRON, np.int32), energy=np.full(n, 50.0), vol=np.zeros(n, np.int32),
              pos=np.zeros((n, 3)), dir=np.tile([0.0, 0.0, 1.0], (n, 1)), nlam=np.full(n, 1.0),
              key=np.arange(3 * n, dtype=np.uint32).reshape(n, 3), nstep=np.zeros(n, np.uint32),
              event=np.zeros(n, np.uint32))
    for r in w.step_tracks(wl.seed, st):
        assert r.out[0].w == 1.0


def test_scattered_showers_conserve_energy(orc):
    wl = W.calorimeter(40)
    opts = W.Options(production_cut=0.07, msc=1)
    r = orc.World(wl.materials, opts, wl.geometry).run_events(wl.seed, wl.events)
    L = r["ledger"]
    bal = (L[:, 0] - (r["dep"].sum(1) + L[:, 1] + L[:, 2] + 2 * ME * (L[:, 3] - L[:, 4]))) / L[:, 0]
    assert np.abs(bal).max() < 1e-12
    # scattering spreads the showers sideways: more energy leaves through the walls
    r0 = orc.World(wl.materials, W.Options(production_cut=0.07), wl.geometry).run_events(wl.seed, wl.events)
    assert L[:, 1].sum() > r0["ledger"][:, 1].sum()
