"""Pins of the oracle's charged-track propagation in a uniform field (CPU): the RK4
path against the analytic helix, the boundary crossing against the exact
helix-cylinder intersection, the substep cap of a vacuum step and the looper rule
(forty capped vacuum steps in a row), and energy conservation of barrel events with
the field on."""
import math

import numpy as np
import pytest
from scipy import optimize

import workloads as W

ME = 0.51099895


def _vacuum_world(orc, radii, half_z=1.0e6, bz=1.0, tol=1.0e-5):
    n = len(radii) - 1
    g = W.Geometry(1, np.array(radii, np.float64), np.full(n, -1, np.int32),
                   np.zeros(n, np.int32), 1, half_z=half_z, bz=bz, field_tol=tol)
    return orc.World([W.LEAD], W.Options(production_cut=0.07), g)


def _helix(p0, d0, kappa, s):
    """Exact solution of dr/ds = d, dd/ds = kappa (d_y, -d_x, 0)."""
    c, sn = math.cos(kappa * s), math.sin(kappa * s)
    dx, dy, dz = d0
    x = p0[0] + (dx * sn + dy * (1 - c)) / kappa
    y = p0[1] + (-dx * (1 - c) + dy * sn) / kappa
    return np.array([x, y, p0[2] + dz * s]), np.array([dx * c + dy * sn, -dx * sn + dy * c, dz])


def test_curvature_constant(orc):
    # textbook: R [m] = p_T [GeV/c] / (0.299792458 B [T])
    k = orc.closed("field_kappa", 1.0, 1.0, 1000.0)
    assert 1.0 / k == pytest.approx(100.0 / 0.299792458, rel=1e-12)
    assert orc.closed("field_kappa", -1.0, 2.0, 500.0) == pytest.approx(-4.0 * k, rel=1e-12)


@pytest.mark.parametrize("p_mev,theta", [(100.0, 1.0), (20.0, 0.3), (1000.0, 1.4)])
def test_rk4_path_follows_helix(orc, p_mev, theta):
    w = _vacuum_world(orc, [0.0, 1.0e6])
    kappa = orc.closed("field_kappa", -1.0, 1.0, p_mev)
    d0 = [math.sin(theta), 0.0, math.cos(theta)]
    # the matter rules (no substep cap below 10^4): the path runs to s_max
    st, s, pos, d, nx = w.field_move(0, kappa, 400.0, 0, [0.0, 0.0, 0.0], d0)
    assert st == 0 and s == pytest.approx(400.0, rel=1e-12)
    pe, de = _helix([0.0, 0.0, 0.0], d0, kappa, s)
    assert np.abs(np.array(pos) - pe).max() < 2e-3  # accumulated from substeps of <= 1e-5 cm
    assert np.abs(np.array(d) - de).max() < 1e-5
    assert abs(np.linalg.norm(d) - 1.0) < 1e-14


@pytest.mark.parametrize("p_mev,theta,phi", [(200.0, 1.2, 0.3), (150.0, 0.8, 2.0)])
def test_boundary_crossing_on_cylinder(orc, p_mev, theta, phi):
    R = 50.0
    w = _vacuum_world(orc, [0.0, R, 100.0])
    kappa = orc.closed("field_kappa", 1.0, 1.0, p_mev)
    p0 = [1.0, -2.0, 3.0]
    d0 = [math.sin(theta) * math.cos(phi), math.sin(theta) * math.sin(phi), math.cos(theta)]
    st, s, pos, d, nx = w.field_move(0, kappa, 1.0e9, 1, p0, d0)
    assert st == 1 and nx == 1
    assert math.hypot(pos[0], pos[1]) == pytest.approx(R, abs=1e-9)
    f = lambda t: math.hypot(*_helix(p0, d0, kappa, t)[0][:2]) - R
    s_true = optimize.brentq(f, 1e-6, 200.0, xtol=1e-14)
    pt, dt = _helix(p0, d0, kappa, s_true)
    # the crossing sits on a chord whose sagitta is within the tolerance
    assert abs(s - s_true) < 1e-3
    assert np.abs(np.array(pos) - pt).max() < 1e-3
    assert np.abs(np.array(d) - dt).max() < 1e-4


def test_vacuum_step_cap_and_looper(orc):
    w = _vacuum_world(orc, [0.0, 50.0, 100.0])
    kappa = orc.closed("field_kappa", -1.0, 1.0, math.sqrt(1.0 * (1.0 + 2 * ME)))
    st, s, pos, d, nx = w.field_move(0, kappa, 1.0e9, 1, [10.0, 0.0, 0.0], [0.0, 1.0, 0.0])
    assert st == 3  # a 1 MeV electron circling in vacuum: the step ends on its substep cap
    assert math.hypot(pos[0], pos[1]) < 11.0
    # in the step: capped vacuum steps go on (limiter 4) until the 40th in a row,
    # which kills the track (limiter 3); a boundary resets the count
    wl = W.barrel(1)
    wo = orc.World(wl.materials, wl.options, wl.geometry)
    n = 3
    st_in = dict(species=np.full(n, W.ELECTRON, np.int32), energy=np.full(n, 1.0),
                 vol=np.zeros(n, np.int32), pos=np.array([[1.0, 0, 0]] * n),
                 dir=np.array([[0, 1.0, 0]] * n), nlam=np.full(n, 1.0),
                 key=np.arange(3 * n, dtype=np.uint32).reshape(n, 3), nstep=np.zeros(n, np.uint32),
                 event=np.zeros(n, np.uint32), vcap=np.array([0, 38, 39], np.uint32))
    res = wo.step_tracks(wl.seed, st_in)
    assert [r.limiter for r in res] == [4, 4, 3]
    assert res[0].parent_alive and res[0].out[0].vac_caps == 1
    assert res[1].parent_alive and res[1].out[0].vac_caps == 39
    assert not res[2].parent_alive and res[2].killed == 1.0


def test_barrel_events_conserve_energy(orc):
    wl = W.barrel(4)
    ev = wl.events
    ev.energy[:] = np.array([1000.0, 2000.0, 1500.0, 800.0])
    w = orc.World(wl.materials, wl.options, wl.geometry)
    r = w.run_events(wl.seed, ev)
    L = r["ledger"]
    bal = L[:, 0] - (r["dep"].sum(1) + L[:, 1] + L[:, 2] + 2 * ME * (L[:, 3] - L[:, 4]))
    assert np.abs(bal / L[:, 0]).max() < 1e-12
    assert r["dep"].sum() > 0
