"""Pins of the oracle's final-state kinematics (CPU).

Interactions are forced in `or_step` by giving states a tiny number of
interaction lengths left (the step ends at once in a discrete interaction), with
random keys so that the process selection and the samplers run on many streams.
Every product is then checked against physics the oracle does not use in that
form:

* momentum conservation, vector by vector, with the target electron at rest
  (Compton, Moller, Bhabha, annihilation in flight): |sum p_out - p_in| is at the
  rounding level of p_in;
* polar angles of the two-body final states, written here from energy and
  momentum conservation (the Compton relation, and the law of cosines for the
  Moller/Bhabha pair);
* products along the parent where the model says so (pair, brems photon,
  photo-electron) and energy bookkeeping of every process;
* the rotation itself: the angle to the input is acos(c), distinct azimuths are
  related as a rotation about the input, the lab-frame branch along +-z behaves
  the same, and azimuths of real products are uniform (chi-square);
* annihilation at rest: two photons of m c^2, exactly back to back, cos(theta)
  and phi uniform (chi-square).
"""
import math

import numpy as np
import pytest
from scipy import stats

import workloads as W

ME = 0.51099895
TOL = 1e-12


def _world(orc):
    wl = W.calorimeter(1)
    return wl, orc.World(wl.materials, wl.options, wl.geometry)


def _forced_states(n, species, e_lo, e_hi, seed, z=0.1, direction=None):
    """States in the middle of the first Pb slab (z = 0.1, far from every surface
    compared with the step), about to interact: interaction lengths left 1e-12."""
    rng = np.random.default_rng(seed)
    T = np.exp(np.log(e_lo) + rng.random(n) * np.log(e_hi / e_lo))
    if direction is None:
        cost = 2 * rng.random(n) - 1
        phi = 2 * np.pi * rng.random(n)
        st = np.sqrt(1 - cost ** 2)
        d = np.stack([st * np.cos(phi), st * np.sin(phi), cost], 1)
    else:
        d = np.tile(np.asarray(direction, np.float64), (n, 1))
    pos = np.zeros((n, 3))
    pos[:, 2] = z
    return dict(species=np.full(n, species, np.int32), energy=T, vol=np.zeros(n, np.int32),
                pos=pos, dir=d, nlam=np.full(n, 1e-12),
                key=rng.integers(0, 2 ** 32, size=(n, 3), dtype=np.uint64).astype(np.uint32),
                nstep=rng.integers(0, 1000, n).astype(np.uint32), event=np.zeros(n, np.uint32))


def _vec(t):
    return np.array([t.u, t.v, t.w])


def _p(T):
    return math.sqrt(T * (T + 2 * ME))


def _results(orc, species, e_lo, e_hi, n=4000, seed=1, **kw):
    wl, w = _world(orc)
    st = _forced_states(n, species, e_lo, e_hi, seed, **kw)
    res = w.step_tracks(wl.seed, st)
    for r in res:
        assert r.limiter == 1  # every forced state interacts
    return st, res


def _unit(v):
    return abs(np.linalg.norm(v) - 1.0) <= 1e-14


def _azimuth(d_in, d_out):
    """Azimuth of d_out about d_in in a frame built here from a fixed reference axis."""
    ref = np.array([1.0, 0.0, 0.0]) if abs(d_in[0]) < 0.9 else np.array([0.0, 1.0, 0.0])
    e1 = ref - d_in * (ref @ d_in)
    e1 /= np.linalg.norm(e1)
    e2 = np.cross(d_in, e1)
    return math.atan2(d_out @ e2, d_out @ e1)


def _uniform_chi2(x, lo, hi, bins=20):
    h, _ = np.histogram(x, bins=bins, range=(lo, hi))
    return stats.chisquare(h).pvalue


# --------------------------------------------------------------------------- rotation

def test_rotation_angle_and_azimuth_geometry(orc):
    rng = np.random.default_rng(5)
    for _ in range(400):
        cost = 2 * rng.random() - 1
        phi = 2 * np.pi * rng.random()
        st = math.sqrt(1 - cost ** 2)
        d = np.array([st * math.cos(phi), st * math.sin(phi), cost])
        c = 2 * rng.random() - 1
        s = math.sqrt(1 - c * c)
        p1, p2 = 2 * np.pi * rng.random(2)
        o1, o2 = orc.rotate(d, c, p1), orc.rotate(d, c, p2)
        assert _unit(o1) and _unit(o2)
        assert abs(o1 @ d - c) <= 1e-14  # polar angle acos(c) to the input
        # two azimuths on the same cone: o1.o2 = c^2 + s^2 cos(phi1 - phi2)
        assert abs(o1 @ o2 - (c * c + s * s * math.cos(p1 - p2))) <= 1e-14
        # a right-handed turn: the azimuth of o2 minus that of o1 is phi2 - phi1
        da = _azimuth(d, o2) - _azimuth(d, o1)
        if s > 1e-6:
            assert abs(math.remainder(da - (p2 - p1), 2 * math.pi)) <= 1e-9 / s


@pytest.mark.parametrize("w", [1.0, -1.0])
def test_rotation_lab_frame_branch(orc, w):
    d = np.array([0.0, 0.0, w])
    for c in (-0.9, -0.2, 0.0, 0.5, 0.99):
        s = math.sqrt(1 - c * c)
        for phi in (0.0, 1.0, 2.5, 4.0, 6.0):
            o = orc.rotate(d, c, phi)
            assert _unit(o) and abs(o @ d - c) <= 1e-15
            o2 = orc.rotate(d, c, phi + 0.7)
            assert abs(o @ o2 - (c * c + s * s * math.cos(0.7))) <= 1e-14
    # just off the axis the general branch takes over continuously
    eps = 1e-9
    dn = np.array([eps, 0.0, w * math.sqrt(1 - eps * eps)])
    o = orc.rotate(dn, 0.3, 1.2)
    assert abs(o @ dn - 0.3) <= 1e-14


# --------------------------------------------------------------------------- photons

def test_compton_kinematics(orc):
    st, res = _results(orc, W.GAMMA, 0.05, 100.0, n=5000, seed=11)
    n_checked, az = 0, []
    for i, r in enumerate(res):
        if r.process != 0:
            continue
        E = st["energy"][i]
        d_in = st["dir"][i]
        outs = [r.out[k] for k in range(r.n_out)]
        gam = [t for t in outs if t.species == W.GAMMA]
        ele = [t for t in outs if t.species == W.ELECTRON]
        assert len(ele) <= 1 and len(gam) <= 1
        if not gam or not ele:  # one product below the tracking cut: deposited
            E1 = gam[0].T if gam else None
            Te = ele[0].T if ele else None
            parts = [x for x in (E1, Te) if x is not None]
            assert abs(sum(parts) + r.dep - E) <= TOL * E
            continue
        g, e = gam[0], ele[0]
        d1, de = _vec(g), _vec(e)
        assert _unit(d1) and _unit(de)
        assert abs(g.T + e.T - E) <= TOL * E and r.dep == 0.0
        # Compton relation between the scattered energy and the photon's polar angle
        k = E / ME
        assert abs(g.T - E / (1 + k * (1 - d1 @ d_in))) <= 1e-10 * E
        # momentum conservation with the electron at rest
        miss = E * d_in - (g.T * d1 + _p(e.T) * de)
        assert np.abs(miss).max() <= 1e-11 * E
        az.append(_azimuth(d_in, d1))
        n_checked += 1
    assert n_checked > 800
    assert _uniform_chi2(az, -math.pi, math.pi) > 1e-3


def test_photoelectric_and_pair_products_follow_the_photon(orc):
    st, res = _results(orc, W.GAMMA, 0.03, 200.0, n=6000, seed=12)
    seen = {1: 0, 2: 0}
    for i, r in enumerate(res):
        E, d_in = st["energy"][i], st["dir"][i]
        if r.process == 1:  # photo-electron with all of E along the photon
            assert r.n_out == 1 and r.out[0].species == W.ELECTRON
            assert r.out[0].T == E and np.array_equal(_vec(r.out[0]), d_in)
            seen[1] += 1
        elif r.process == 2:
            assert r.n_pair == 1 and r.parent_alive == 0
            tot = r.dep + sum(r.out[k].T for k in range(r.n_out))
            gam = sum(1 for k in range(r.n_out) if r.out[k].species == W.GAMMA)
            # e- and e+ share E - 2m; a positron below the tracking cut annihilates at rest
            assert abs(tot - (E - 2 * ME) - 2 * ME * r.n_annih) <= TOL * E
            for k in range(r.n_out):
                if r.out[k].species != W.GAMMA:
                    assert np.array_equal(_vec(r.out[k]), d_in)
            assert gam == 2 * r.n_annih
            seen[2] += 1
    assert seen[1] > 100 and seen[2] > 300


# --------------------------------------------------------------------------- e-/e+

def _two_body_delta(orc, species, seed):
    st, res = _results(orc, species, 2.5, 100.0, n=8000, seed=seed)
    n_checked, az = 0, []
    for i, r in enumerate(res):
        if r.process != 0:
            continue
        d_in = st["dir"][i]
        outs = [r.out[k] for k in range(r.n_out)]
        delta = [t for t in outs if t.species == W.ELECTRON and t.nstep == 0]
        parent = [t for t in outs if t.species == species and t.nstep > 0]
        assert len(delta) == 1
        dl = delta[0]
        if not parent:  # a positron left below the tracking cut: deposited, at rest
            assert species == W.POSITRON
            continue
        pa = parent[0]
        T1 = pa.T + dl.T  # post-step kinetic energy of the projectile
        dd, dp = _vec(dl), _vec(pa)
        assert _unit(dd) and _unit(dp)
        assert dl.T <= (0.5 if species == W.ELECTRON else 1.0) * T1 * (1 + 1e-15)
        # law of cosines from energy and momentum conservation, target at rest
        P1, Pd, Pp = _p(T1), _p(dl.T), _p(pa.T)
        cos_delta = (P1 * P1 + Pd * Pd - Pp * Pp) / (2 * P1 * Pd)
        assert abs(dd @ d_in - cos_delta) <= 1e-9
        miss = P1 * d_in - (Pd * dd + Pp * dp)
        assert np.abs(miss).max() <= 1e-11 * P1
        az.append(_azimuth(d_in, dd))
        n_checked += 1
    assert n_checked > 300
    assert _uniform_chi2(az, -math.pi, math.pi) > 1e-3


def test_moller_kinematics(orc):
    _two_body_delta(orc, W.ELECTRON, 21)


def test_bhabha_kinematics(orc):
    _two_body_delta(orc, W.POSITRON, 22)


def test_brems_photon_along_parent(orc):
    for sp, seed in ((W.ELECTRON, 31), (W.POSITRON, 32)):
        st, res = _results(orc, sp, 1.0, 1e4, n=3000, seed=seed)
        n = 0
        for i, r in enumerate(res):
            if r.process != 1:
                continue
            d_in = st["dir"][i]
            outs = [r.out[k] for k in range(r.n_out)]
            # the brems photon is the last product (at-rest photons of a positron left
            # below the tracking cut come before it)
            ph = [outs[-1]]
            assert ph[0].species == W.GAMMA
            pa = [t for t in outs if t.species == sp and t.nstep > 0]
            assert np.array_equal(_vec(ph[0]), d_in)
            T_in = st["energy"][i]
            if pa:  # the parent keeps its direction and the rest of its energy
                assert np.array_equal(_vec(pa[0]), d_in)
                assert abs(ph[0].T + pa[0].T + r.dep - T_in) <= TOL * T_in
                assert r.dep <= 1e-9 * T_in  # only the continuous loss of the tiny step
            n += 1
        assert n > 300


def test_annihilation_in_flight_kinematics(orc):
    st, res = _results(orc, W.POSITRON, 0.05, 20.0, n=20000, seed=41)
    n_checked, az = 0, []
    for i, r in enumerate(res):
        if r.process != 2:
            continue
        d_in = st["dir"][i]
        assert r.n_annih == 1 and r.parent_alive == 0 and r.n_out == 2
        g1, g2 = r.out[0], r.out[1]
        assert g1.species == W.GAMMA and g2.species == W.GAMMA
        T1 = g1.T + g2.T - 2 * ME
        d1, d2 = _vec(g1), _vec(g2)
        assert _unit(d1) and _unit(d2)
        # the photons carry the positron's momentum (the electron is at rest)
        miss = _p(T1) * d_in - (g1.T * d1 + g2.T * d2)
        assert np.abs(miss).max() <= 1e-11 * (T1 + 2 * ME)
        az.append(_azimuth(d_in, d1))
        n_checked += 1
    assert n_checked > 200
    assert _uniform_chi2(az, -math.pi, math.pi, bins=10) > 1e-3


def test_annihilation_at_rest_back_to_back_isotropic(orc):
    # positrons that range out in one step annihilate at rest
    wl, w = _world(orc)
    n = 6000
    st = _forced_states(n, W.POSITRON, 0.0101, 0.0102, 51, direction=(0.0, 0.0, 1.0))
    st["nlam"][:] = 50.0  # no discrete interaction: the step ends by range-out
    res = w.step_tracks(wl.seed, st)
    cos_z, phis = [], []
    for i, r in enumerate(res):
        assert r.n_annih == 1 and r.parent_alive == 0 and r.n_out == 2
        g1, g2 = r.out[0], r.out[1]
        assert g1.species == g2.species == W.GAMMA and g1.T == ME and g2.T == ME
        d1, d2 = _vec(g1), _vec(g2)
        assert _unit(d1) and np.array_equal(d1, -d2)
        assert abs(r.dep - st["energy"][i]) <= TOL
        cos_z.append(d1[2])
        phis.append(math.atan2(d1[1], d1[0]))
    assert _uniform_chi2(cos_z, -1, 1) > 1e-3
    assert _uniform_chi2(phis, -math.pi, math.pi) > 1e-3
