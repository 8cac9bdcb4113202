"""Pins of the oracle's quadric-surface cell navigation (CPU only).

The navigation (paper Sec. 2.3, ORANGE: cells bounded by quadric surfaces, single
level) is checked against things that do not come from it:
* the slab calorimeter written as quadric cells transports every event exactly as
  the oracle's own closed-form slab navigation (deposits, ledger and step counts
  bitwise equal);
* exit distances equal the textbook ray-sphere, ray-cylinder and ray-cone roots;
* for random rays in the module, the point just before the computed boundary is
  still in the start cell and the point just after it is in the cell entered, by
  membership predicates written here from the geometry's description;
* located cells agree with those predicates, and the fraction of uniform points
  located in each cell matches the cells' analytic volumes (chi-square);
* module events conserve energy to 1e-12.
"""
import math

import numpy as np
import pytest

import workloads as W

ME = 0.51099895


def test_slab_calorimeter_as_quadric_cells_is_the_same_transport(orc):
    wl = W.calorimeter(150)
    slab = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, wl.events)
    csg = orc.World(wl.materials, wl.options, W.calorimeter_csg()).run_events(wl.seed, wl.events)
    assert np.array_equal(slab["dep"], csg["dep"])
    assert np.array_equal(slab["ledger"], csg["ledger"])
    assert np.array_equal(slab["steps"], csg["steps"])


def _unit(rng, n):
    c = 2 * rng.random(n) - 1
    p = 2 * np.pi * rng.random(n)
    s = np.sqrt(1 - c * c)
    return np.stack([s * np.cos(p), s * np.sin(p), c], 1)


def test_exit_distances_equal_textbook_roots(orc):
    rng = np.random.default_rng(3)
    R = 7.5
    sph = W.sphere(R, (1.0, -2.0, 0.5))
    cyl = W.cylinder(0, 3.0)
    cone = W.cone_z(0.3)
    for _ in range(300):
        d = _unit(rng, 1)[0]
        # from inside the sphere (side -1): t = -(q.d) + sqrt((q.d)^2 - |q|^2 + R^2), q = p - c
        q = rng.normal(size=3) * 2.0
        p = q + np.array([1.0, -2.0, 0.5])
        if q @ q >= R * R:
            continue
        qd = q @ d
        t = -qd + math.sqrt(qd * qd - (q @ q - R * R))
        assert abs(orc.csg_exit(sph, p, d, -1) - t) <= 1e-12 * max(t, 1.0)
        # from outside the sphere moving away: never
        far = p + 3 * R * d
        assert orc.csg_exit(sph, far, d, 1) == math.inf
        # entering from outside (side +1) along -d toward the centre: the near root
        qf = far - np.array([1.0, -2.0, 0.5])
        b = qf @ (-d)
        tn = -b - math.sqrt(b * b - (qf @ qf - R * R))
        assert abs(orc.csg_exit(sph, far, -d, 1) - tn) <= 1e-12 * max(tn, 1.0)
    for _ in range(300):
        d = _unit(rng, 1)[0]
        p = np.array([rng.uniform(-5, 5), *rng.uniform(-2, 2, 2)])
        if p[1] ** 2 + p[2] ** 2 >= 9.0 or d[1] ** 2 + d[2] ** 2 < 1e-6:
            continue
        a = d[1] ** 2 + d[2] ** 2
        b = p[1] * d[1] + p[2] * d[2]
        c = p[1] ** 2 + p[2] ** 2 - 9.0
        t = (-b + math.sqrt(b * b - a * c)) / a
        assert abs(orc.csg_exit(cyl, p, d, -1) - t) <= 1e-11 * max(t, 1.0)
    # a ray along the cone's axis from inside the lower nappe never leaves it; a ray
    # across it leaves where x^2 + y^2 = (0.3 z)^2
    assert orc.csg_exit(cone, [0, 0, -15.0], [0, 0, -1.0], -1) == math.inf
    p, d = np.array([0.0, 0.0, -15.0]), np.array([1.0, 0.0, 0.0])
    assert abs(orc.csg_exit(cone, p, d, -1) - 4.5) <= 1e-12 * 4.5
    # a tangent ray does not cross; a plane gives the slab formula exactly
    assert orc.csg_exit(W.sphere(2.0), [-5.0, 2.0, 0.0], [1.0, 0.0, 0.0], 1) == math.inf
    pl = W.plane(2, 3.2)
    for z, w in ((1.0, 0.3), (3.1, 0.9), (-4.0, 0.01)):
        assert orc.csg_exit(pl, [0.0, 0.0, z], [0.0, math.sqrt(1 - w * w), w], -1) == (3.2 - z) / w


# membership written from the module's description (not from its surface list)
def _module_cell(p):
    x, y, z = p
    r2 = x * x + y * y + z * z
    if max(abs(x), abs(y), abs(z)) > 20:
        return -1
    if r2 < 64:
        if abs(x) < 6 and y * y + z * z < 9:
            return 0
        if x < -6:
            return 2
        if x > 6:
            return 3
        return 1
    if r2 < 100:
        return 4
    if z > -10:
        return 5
    return 7 if x * x + y * y < 0.09 * z * z else 6


def _near_surface(p, eps):
    x, y, z = p
    r = math.sqrt(x * x + y * y + z * z)
    vals = [abs(abs(x) - 20), abs(abs(y) - 20), abs(abs(z) - 20), abs(r - 10), abs(r - 8),
            abs(math.sqrt(y * y + z * z) - 3), abs(abs(x) - 6), abs(z + 10),
            abs(math.sqrt(x * x + y * y) - 0.3 * abs(z))]
    return min(vals) < eps


def test_module_locate_and_boundary_crossings(orc):
    wl = W.csg_module(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    rng = np.random.default_rng(11)
    pts = rng.uniform(-20, 20, (3000, 3))
    dirs = _unit(rng, 3000)
    checked = 0
    for p, d in zip(pts, dirs):
        if _near_surface(p, 1e-6):
            continue
        k = w.locate(p, d)
        assert k == _module_cell(p), (p, k)
        s, nxt = w.distance(k, p, d)
        assert math.isfinite(s) and s > 0
        after = p + (s + 1e-4) * d  # just past the boundary (thinnest cell: 2 cm)
        for f in np.linspace(0.0, 1.0, 64)[1:-1]:
            q = p + f * s * d
            if not _near_surface(q, 1e-9):
                assert _module_cell(q) == k
        if not _near_surface(after, 1e-6):
            assert _module_cell(after) == nxt, (p, d, k, s, nxt)
            checked += 1
    assert checked > 2000


def test_module_cell_volumes(orc):
    wl = W.csg_module(1)
    w = orc.World(wl.materials, wl.options, wl.geometry)
    rng = np.random.default_rng(5)
    n = 120_000
    pts = rng.uniform(-20, 20, (n, 3))
    counts = np.zeros(8)
    d = np.array([0.0, 0.0, 1.0])
    for p in pts:
        counts[w.locate(p, d)] += 1
    cap = math.pi * 2.0 ** 2 * (3 * 8 - 2) / 3  # sphere of radius 8 beyond |x| = 6
    rod = math.pi * 9 * 12
    v8, v10 = 4 / 3 * math.pi * 512, 4 / 3 * math.pi * 1000
    channel = math.pi * 0.09 / 3 * (20 ** 3 - 10 ** 3)
    vol = np.array([rod, v8 - 2 * cap - rod, cap, cap, v10 - v8, 64000 - 16000 - v10,
                    16000 - channel, channel])
    expected = n * vol / 64000
    chi2 = ((counts - expected) ** 2 / expected).sum()
    assert abs(vol.sum() - 64000) < 1e-9
    assert chi2 < 24.3  # 7 degrees of freedom, p = 0.001


def test_module_events_conserve_energy(orc):
    wl = W.csg_module(60)
    r = orc.World(wl.materials, wl.options, wl.geometry).run_events(wl.seed, wl.events)
    L = r["ledger"]
    bal = (L[:, 0] - (r["dep"].sum(1) + L[:, 1] + L[:, 2] + 2 * ME * (L[:, 3] - L[:, 4]))) / L[:, 0]
    assert np.abs(bal).max() < 1e-12
    assert (L[:, 2] == 0).all()  # no track stuck at a surface until the step cap
    assert (r["dep"].sum(0) > 0)[:7].all()  # every material cell is reached
