"""Transport-level pins of the oracle (CPU): narrow-beam attenuation, CSDA range,
per-event energy conservation, geometry distances, and reproducibility."""
import math

import numpy as np
import pytest

import workloads as W

ME = 0.51099895


def _slab_world(orc, thickness, opts, mats=(W.LEAD,), half=1e6):
    g = W.Geometry(0, np.array([0.0, thickness]), np.array([0], np.int32), np.array([0], np.int32),
                   1, half_x=half, half_y=half)
    return orc.World(list(mats), opts, g), g


@pytest.mark.parametrize("E", [0.1, 1.0, 10.0, 1000.0])
def test_narrow_beam_uncollided_fraction(orc, E):
    """Photons entering a slab of thickness 1/mu at normal incidence leave through the back
    without interacting with probability exp(-mu t) = 1/e, mu the tabulated attenuation."""
    opts = W.Options(charged_local=1)
    w, g = _slab_world(orc, 1.0, opts)
    mu = sum(w.interp(0, 0, q, E) for q in range(3))
    if E <= 2 * ME:
        mu -= w.interp(0, 0, 2, E)
    t = 1.0 / mu
    w, g = _slab_world(orc, t, opts)
    n = 60000
    rng = np.random.default_rng(3)
    st = dict(species=np.zeros(n, np.int32), energy=np.full(n, E), vol=np.zeros(n, np.int32),
              pos=np.zeros((n, 3)), dir=np.tile([0.0, 0.0, 1.0], (n, 1)), nlam=np.full(n, -1.0),
              key=rng.integers(0, 2 ** 32, (n, 3), dtype=np.uint64).astype(np.uint32),
              nstep=np.zeros(n, np.uint32), event=np.zeros(n, np.uint32))
    res = w.step_tracks(1, st)
    through = sum(1 for r in res if r.escaped and r.limiter == 0 and r.esc == E)
    f = through / n
    p = math.exp(-1.0)
    assert abs(f - p) < 4.5 * math.sqrt(p * (1 - p) / n), f


@pytest.mark.parametrize("species,T0", [(1, 1.0), (1, 50.0), (2, 5.0)])
def test_csda_range(orc, species, T0):
    """With no discrete processes an e-/e+ travels exactly R(T0) - R(T_cut) before it stops,
    and the tabulated range matches the integral of dT/S(T) within its interpolation error."""
    opts = W.Options(production_cut=0.07, ionisation=0, brems=0, annihilation=0)
    w, g = _slab_world(orc, 1e6, opts)
    st = dict(species=np.array([species], np.int32), energy=np.array([T0]), vol=np.zeros(1, np.int32),
              pos=np.array([[0.0, 0.0, 1.0]]), dir=np.array([[0.0, 0.0, 1.0]]), nlam=np.array([-1.0]),
              key=np.array([[1, 2, 3]], np.uint32), nstep=np.zeros(1, np.uint32),
              event=np.zeros(1, np.uint32))
    path = 0.0
    dep = 0.0
    for _ in range(100000):
        r = w.step_tracks(7, st)[0]
        path += r.step_len
        dep += r.dep
        if not r.parent_alive:
            break
        t = r.out[0]
        st = dict(species=np.array([t.species], np.int32), energy=np.array([t.T]),
                  vol=np.array([t.vol], np.int32), pos=np.array([[t.x, t.y, t.z]]),
                  dir=np.array([[t.u, t.v, t.w]]), nlam=np.array([t.nlam]),
                  key=np.array([list(t.key)], np.uint32), nstep=np.array([t.nstep], np.uint32),
                  event=np.zeros(1, np.uint32))
    else:
        pytest.fail("track did not stop")
    R0 = w.interp(0, species, 3, T0)
    assert path == pytest.approx(R0 - w.range_at_cut(0, species), rel=1e-12)
    assert dep == pytest.approx(T0, rel=1e-12)
    # range table vs direct integral of dT/S with the full (unrestricted) loss
    from scipy import integrate
    Z, A, rho, I = W.LEAD
    n_el = Z * rho * 6.02214076e23 / A
    X0 = orc.closed("radiation_length", Z, A, rho)
    S = lambda T: orc.closed("scol", species - 1, n_el, I, T, 1e9) + orc.closed("brems_Srad", X0, T, T)
    R = integrate.quad(lambda l: math.exp(l) / S(math.exp(l)), math.log(0.01), math.log(T0),
                       epsrel=1e-12)[0]
    assert path == pytest.approx(R, rel=2e-3)


def _ledger_residual(r):
    L = r["ledger"]
    dep = r["dep"].sum(1)
    return (L[:, 0] - (dep + L[:, 1] + L[:, 2] + 2 * ME * (L[:, 3] - L[:, 4]))) / L[:, 0]


def test_energy_conservation_photon_cube(orc):
    wl = W.photon_cube(3000)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    r = w.run_events(wl.seed, wl.events, esc_hist=True)
    assert np.abs(_ledger_residual(r)).max() < 1e-12
    # most 10 MeV photons are absorbed in 13.6 mean free paths of lead
    assert r["dep"].sum() / r["ledger"][:, 0].sum() > 0.9
    assert r["esc_hist"].sum() > 0


def _life_bounds(life):
    """Per species, the least and greatest total step count a steps-per-track histogram allows."""
    b = np.arange(life.shape[1])
    lo = np.where(b == 0, 0, 2.0 ** (b - 1))
    hi = np.where(b == 0, 0, 2.0 ** b - 1)
    life = np.asarray(life, np.float64)
    top = np.where(life[:, -1] > 0, np.inf, 0.0)  # the last bin has no upper end
    return life @ lo, life[:, :-1] @ hi[:-1] + top


def test_life_bins_are_bit_lengths(orc):
    L = orc.lib()
    for n in list(range(0, 70)) + [2 ** k + d for k in range(6, 20) for d in (-1, 0, 1)]:
        assert L.or_life_bin(n) == min(int(n).bit_length(), orc.LIFE_BINS - 1), n


@pytest.mark.parametrize("name", ["photon_cube", "calorimeter"])
def test_steps_per_track_histogram(orc, name):
    """Every track ends once; only a primary born outside takes no step; the histogram
    bounds each species' step count."""
    wl = W.photon_cube(500) if name == "photon_cube" else W.calorimeter(6)
    ev = wl.events
    # move a tenth of the primaries outside the world, heading away from it
    out = np.arange(ev.n_primaries) % 10 == 3
    ev.pos[out] = [0.0, 0.0, -1e4]
    ev.dir[out] = [0.0, 0.0, -1.0]
    r = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, ev, life_hist=True)
    life = r["life_hist"]
    assert np.array_equal(life.sum(1), r["tracks"].astype(np.float64))
    born_out = np.bincount(ev.species[out], minlength=3)
    assert np.array_equal(life[:, 0], born_out.astype(np.float64))
    lo, hi = _life_bounds(life)
    assert (lo <= r["steps"]).all() and (r["steps"] <= hi).all(), (lo, r["steps"], hi)
    assert life[:, 1:].sum() > 0


def test_energy_conservation_calorimeter(orc):
    wl = W.calorimeter(40)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    r = w.run_events(wl.seed, wl.events)
    assert np.abs(_ledger_residual(r)).max() < 1e-12
    assert (r["ledger"][:, 3] > 0).all()  # every 1 GeV shower converts photons
    # the longitudinal profile peaks a few radiation lengths deep (t_max ~ ln(E/Ec) - 1/2)
    layers = r["dep"].reshape(40, 50, 2).sum(2).mean(0)
    assert 3 <= int(np.argmax(layers)) <= 14


def test_events_independent_of_batch_order(orc):
    wl = W.calorimeter(6)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    a = w.run_events(wl.seed, wl.events)
    rev = wl.events.subset(np.arange(5, -1, -1))
    b = w.run_events(wl.seed, rev)
    assert np.array_equal(a["dep"], b["dep"][::-1])
    c = w.run_events(wl.seed + 1, wl.events)
    assert not np.array_equal(a["dep"], c["dep"])


def test_slab_distances_brute_force(orc):
    wl = W.calorimeter(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    rng = np.random.default_rng(5)
    b = wl.geometry.bounds
    for _ in range(300):
        vol = int(rng.integers(0, 100))
        p = np.array([rng.uniform(-20, 20), rng.uniform(-20, 20), rng.uniform(b[vol], b[vol + 1])])
        c = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * np.pi)
        d = np.array([math.sqrt(1 - c * c) * math.cos(ph), math.sqrt(1 - c * c) * math.sin(ph), c])
        s, nx = w.distance(vol, p, d)
        # march: inside before s, outside after s
        inside = lambda q: abs(q[0]) <= 20 and abs(q[1]) <= 20 and b[vol] <= q[2] <= b[vol + 1]
        assert inside(p + d * s * (1 - 1e-9))
        assert not inside(p + d * (s * (1 + 1e-9) + 1e-12))
        q = p + d * s * (1 + 1e-9) + d * 1e-12
        assert nx == w.locate(q, d)


def test_cylinder_distances_brute_force(orc):
    wl = W.barrel(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    rng = np.random.default_rng(6)
    b = wl.geometry.bounds
    n = len(b) - 1
    for _ in range(300):
        vol = int(rng.integers(0, n))
        r = rng.uniform(b[vol], b[vol + 1])
        a = rng.uniform(0, 2 * np.pi)
        p = np.array([r * math.cos(a), r * math.sin(a), rng.uniform(-300, 300)])
        c = rng.uniform(-1, 1)
        ph = rng.uniform(0, 2 * np.pi)
        d = np.array([math.sqrt(1 - c * c) * math.cos(ph), math.sqrt(1 - c * c) * math.sin(ph), c])
        s, nx = w.distance(vol, p, d)

        def inside(q):
            rr = math.hypot(q[0], q[1])
            return abs(q[2]) <= 300 and b[vol] <= rr <= b[vol + 1]
        assert inside(p + d * s * (1 - 1e-9))
        q = p + d * (s * (1 + 1e-9) + 1e-9)
        assert not inside(q)
        assert nx == w.locate(q, d)
