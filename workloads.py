"""Seeded synthetic inputs shared by the tests, the benchmark and the oracle.

This module only describes *inputs*: material constants, geometry
descriptions, run options and the primaries of each event, generated from
numpy's seeded generator.  It holds none of the transport arithmetic and
imports neither the product package nor the oracle; both of those receive
exactly these arrays.

Workloads (energies MeV, lengths cm):

* ``photon_cube``   -- 10 MeV photons on the +z axis into a 10 cm lead cube
  (Z=82, rho=11.35); Compton + photoelectric + pair; charged secondaries
  deposit locally; tracking cut 10 keV.
* ``calorimeter``   -- electrons at normal incidence on 50 layers of
  2 mm Pb + 5 mm liquid Ar (40 x 40 cm); full e-/e+/photon physics,
  production cut 0.7 mm, tracking cut 10 keV.  1 GeV for the FP64 shower,
  10 GeV for the mixed-precision one.
* ``barrel``        -- concentric cylinders (5 Si layers of 300 um between
  r = 4 and 50 cm, 50 Pb/LAr layers over r = 150-200 cm, |z| <= 300 cm) in a
  uniform 1 T field; mixed e-/e+/photon primaries, log-uniform 1-100 GeV,
  isotropic in |eta| < 1.5.
* ``serving``       -- Poisson arrivals of events with 1-500 primaries of
  mixed species, log-uniform 1-100 GeV, on the calorimeter geometry.
"""
from __future__ import annotations

import dataclasses
from typing import Dict, List, Optional

import numpy as np

GAMMA, ELECTRON, POSITRON = 0, 1, 2

# (Z, A [g/mol], density [g/cm^3], mean excitation energy [MeV])
LEAD = (82.0, 207.2, 11.35, 823.0e-6)
LIQUID_ARGON = (18.0, 39.948, 1.396, 188.0e-6)
SILICON = (14.0, 28.0855, 2.33, 173.0e-6)
IRON = (26.0, 55.845, 7.874, 286.0e-6)
COPPER = (29.0, 63.546, 8.96, 322.0e-6)
TUNGSTEN = (74.0, 183.84, 19.3, 727.0e-6)

TRACKING_CUT = 0.01  # 10 keV


@dataclasses.dataclass
class Options:
    tracking_cut: float = TRACKING_CUT
    production_cut: float = 0.0  # cm; <= 0: thresholds equal the tracking cut
    compton: int = 1
    photoelectric: int = 1
    pair: int = 1
    ionisation: int = 1
    brems: int = 1
    annihilation: int = 1
    charged_local: int = 0
    continuous_loss: int = 1
    step_alpha: float = 0.2
    step_rfinal: float = 0.01
    max_steps: int = 1 << 16
    msc: int = 0  # Gaussian multiple-scattering deflection of e-/e+ (not in the benchmark configs)


@dataclasses.dataclass
class Geometry:
    kind: int  # 0 slabs (z planes), 1 cylinders (radii), 2 quadric-surface cells
    bounds: np.ndarray  # n_vol + 1 float64 (kind 0, 1)
    material: np.ndarray  # n_vol int32 (-1 vacuum)
    tally_bin: np.ndarray  # n_vol int32
    n_bins: int
    half_x: float = 0.0
    half_y: float = 0.0
    half_z: float = 0.0
    bz: float = 0.0
    field_tol: float = 1.0e-5
    # kind 2: surfaces (n_surf x 10 coefficients of
    #   qxx x^2 + qyy y^2 + qzz z^2 + qxy xy + qyz yz + qzx zx + px x + py y + pz z + k)
    # and the faces of each cell: cell k has faces[face_off[k]:face_off[k+1]], each
    # surface * 2 + (1 if the cell lies where f > 0, 0 where f < 0)
    surfaces: Optional[np.ndarray] = None
    face_off: Optional[np.ndarray] = None
    faces: Optional[np.ndarray] = None

    @property
    def n_vol(self) -> int:
        return int(self.material.shape[0])


@dataclasses.dataclass
class Events:
    """Primaries of a batch of events, rows grouped by event."""
    event_ids: np.ndarray  # n_events uint32
    offsets: np.ndarray  # n_events + 1 int64
    species: np.ndarray  # n_prim int32
    energy: np.ndarray  # n_prim float64
    pos: np.ndarray  # n_prim x 3 float64
    dir: np.ndarray  # n_prim x 3 float64
    arrival: Optional[np.ndarray] = None  # seconds, serving only

    @property
    def n_events(self) -> int:
        return int(self.event_ids.shape[0])

    @property
    def n_primaries(self) -> int:
        return int(self.species.shape[0])

    def subset(self, idx) -> "Events":
        idx = np.asarray(idx, dtype=np.int64)
        rows = [np.arange(self.offsets[i], self.offsets[i + 1]) for i in idx]
        rows = np.concatenate(rows) if rows else np.zeros(0, np.int64)
        counts = self.offsets[idx + 1] - self.offsets[idx]
        off = np.zeros(len(idx) + 1, np.int64)
        off[1:] = np.cumsum(counts)
        return Events(self.event_ids[idx].copy(), off, self.species[rows].copy(),
                      self.energy[rows].copy(), self.pos[rows].copy(), self.dir[rows].copy(),
                      None if self.arrival is None else self.arrival[idx].copy())


@dataclasses.dataclass
class Workload:
    name: str
    materials: List[tuple]
    options: Options
    geometry: Geometry
    events: Events
    seed: int
    note: str = ""


def _single_primary_events(n: int, species: int, energy: float, pos, direction,
                           first_id: int = 0) -> Events:
    ids = np.arange(first_id, first_id + n, dtype=np.uint32)
    off = np.arange(n + 1, dtype=np.int64)
    sp = np.full(n, species, np.int32)
    en = np.full(n, energy, np.float64)
    p = np.tile(np.asarray(pos, np.float64), (n, 1))
    d = np.tile(np.asarray(direction, np.float64), (n, 1))
    return Events(ids, off, sp, en, p, d)


def calorimeter_geometry(n_layers: int = 50, pb: float = 0.2, lar: float = 0.5,
                         half_xy: float = 20.0) -> Geometry:
    """Slab stack: layer i is Pb on [i p, i p + pb] then LAr up to (i+1) p, p = pb+lar.
    Tally bin = volume (Pb of layer i -> 2i, LAr -> 2i+1)."""
    pitch = pb + lar
    b = []
    for i in range(n_layers):
        b.append(pitch * i)
        b.append(pitch * i + pb)
    b.append(pitch * n_layers)
    bounds = np.array(b, np.float64)
    mat = np.tile(np.array([0, 1], np.int32), n_layers)
    bins = np.arange(2 * n_layers, dtype=np.int32)
    return Geometry(0, bounds, mat, bins, 2 * n_layers, half_x=half_xy, half_y=half_xy)


def photon_cube(n_events: int = 10_000, energy: float = 10.0, seed: int = 1) -> Workload:
    geom = Geometry(0, np.array([-5.0, 5.0]), np.array([0], np.int32), np.array([0], np.int32),
                    1, half_x=5.0, half_y=5.0)
    opts = Options(production_cut=0.0, charged_local=1)
    ev = _single_primary_events(n_events, GAMMA, energy, (0.0, 0.0, -5.0), (0.0, 0.0, 1.0))
    return Workload("photon_cube", [LEAD], opts, geom, ev, seed,
                    f"{n_events} x {energy} MeV photons into a 10 cm Pb cube")


def calorimeter(n_events: int = 100_000, energy: float = 1000.0, seed: int = 2,
                first_id: int = 0) -> Workload:
    geom = calorimeter_geometry()
    opts = Options(production_cut=0.07)
    ev = _single_primary_events(n_events, ELECTRON, energy, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0),
                                first_id)
    return Workload("calorimeter", [LEAD, LIQUID_ARGON], opts, geom, ev, seed,
                    f"{n_events} x {energy / 1000:g} GeV e- on 50 x (2 mm Pb + 5 mm LAr)")


def material_stack(n_events: int = 200, energy: float = 1000.0, seed: int = 6) -> Workload:
    """Six materials in turn (Pb, Fe, Cu, Si, LAr, W), 30 slabs of 4 mm, 40 x 40 cm;
    electrons at normal incidence from the origin, calorimeter physics.  In FP64 the
    charged-particle tables of six materials (6 x 2 x 200 x 4 doubles = 76.8 KB)
    exceed the 64 KB per-block staging budget of the step kernels, so this workload
    runs their global-memory variant."""
    n_slab = 30
    bounds = np.arange(n_slab + 1, dtype=np.float64) * 0.4
    mat = (np.arange(n_slab) % 6).astype(np.int32)
    geom = Geometry(0, bounds, mat, np.arange(n_slab, dtype=np.int32), n_slab, half_x=20.0,
                    half_y=20.0)
    ev = _single_primary_events(n_events, ELECTRON, energy, (0.0, 0.0, 0.0), (0.0, 0.0, 1.0))
    return Workload("material_stack", [LEAD, IRON, COPPER, SILICON, LIQUID_ARGON, TUNGSTEN],
                    Options(production_cut=0.07), geom, ev, seed,
                    f"{n_events} x {energy / 1000:g} GeV e- on 30 slabs of six materials")


# ---- quadric surfaces (coefficients only) and cells built from them
def plane(axis: int, at: float) -> np.ndarray:
    """f = x_axis - at."""
    q = np.zeros(10)
    q[6 + axis] = 1.0
    q[9] = -at
    return q


def sphere(r: float, center=(0.0, 0.0, 0.0)) -> np.ndarray:
    cx, cy, cz = center
    return np.array([1.0, 1.0, 1.0, 0.0, 0.0, 0.0, -2 * cx, -2 * cy, -2 * cz,
                     cx * cx + cy * cy + cz * cz - r * r])


def cylinder(axis: int, r: float) -> np.ndarray:
    """Infinite circular cylinder of radius r about a coordinate axis through the origin."""
    q = np.zeros(10)
    for a in range(3):
        if a != axis:
            q[a] = 1.0
    q[9] = -r * r
    return q


def cone_z(slope: float) -> np.ndarray:
    """x^2 + y^2 - (slope z)^2: both nappes of a cone about z with its apex at the origin."""
    return np.array([1.0, 1.0, -slope * slope, 0, 0, 0, 0, 0, 0, 0.0])


def _cells(cells):
    """cells: list of lists of (surface, sense) with sense -1 (f < 0) or +1 (f > 0)."""
    off = np.zeros(len(cells) + 1, np.int32)
    faces = []
    for k, c in enumerate(cells):
        faces += [2 * s + (1 if sense > 0 else 0) for s, sense in c]
        off[k + 1] = len(faces)
    return off, np.array(faces, np.int32)


def calorimeter_csg(n_layers: int = 50, pb: float = 0.2, lar: float = 0.5,
                    half_xy: float = 20.0) -> Geometry:
    """The slab calorimeter written as quadric-surface cells: every Pb or LAr slab is
    the cell between two z planes and the four lateral walls.  Faces are listed
    y walls, x walls, then z planes, so that ties go to the walls (y before x) as
    in the slab navigation."""
    slab = calorimeter_geometry(n_layers, pb, lar, half_xy)
    b = slab.bounds
    surf = [plane(1, -half_xy), plane(1, half_xy), plane(0, -half_xy), plane(0, half_xy)]
    surf += [plane(2, z) for z in b]
    cells = [[(0, 1), (1, -1), (2, 1), (3, -1), (4 + i, 1), (5 + i, -1)] for i in range(len(b) - 1)]
    off, faces = _cells(cells)
    return Geometry(2, np.zeros(len(b)), slab.material.copy(), slab.tally_bin.copy(), slab.n_bins,
                    surfaces=np.array(surf), face_off=off, faces=faces)


def csg_module_geometry() -> Geometry:
    """A 40 cm cube of lead holding a silicon spherical shell (8 < r < 10 cm) around
    liquid argon, in which a tungsten rod (radius 3 cm along x, |x| < 6 cm) sits at
    the centre; a conical vacuum channel (x^2 + y^2 < (0.3 z)^2) runs from the face
    z = -20 cm to z = -10 cm.  Spheres, an x-cylinder, a cone and planes; every cell
    is an intersection of half-spaces."""
    surf = [plane(0, -20.0), plane(0, 20.0), plane(1, -20.0), plane(1, 20.0), plane(2, -20.0),
            plane(2, 20.0),                 # 0-5 faces of the cube
            sphere(10.0), sphere(8.0),      # 6, 7
            cylinder(0, 3.0),               # 8
            plane(0, -6.0), plane(0, 6.0),  # 9, 10
            plane(2, -10.0),                # 11
            cone_z(0.3)]                    # 12
    box_sides = [(0, 1), (1, -1), (2, 1), (3, -1)]
    cells = [
        [(8, -1), (9, 1), (10, -1)],                             # 0 tungsten rod
        [(7, -1), (9, 1), (10, -1), (8, 1)],                     # 1 LAr around the rod
        [(7, -1), (9, -1)],                                      # 2 LAr, x < -6
        [(7, -1), (10, 1)],                                      # 3 LAr, x > 6
        [(6, -1), (7, 1)],                                       # 4 Si shell
        box_sides + [(5, -1), (11, 1), (6, 1)],                  # 5 Pb above z = -10
        box_sides + [(4, 1), (11, -1), (12, 1)],                 # 6 Pb below, outside the cone
        box_sides + [(4, 1), (11, -1), (12, -1)],                # 7 vacuum channel
    ]
    off, faces = _cells(cells)
    material = np.array([3, 1, 1, 1, 2, 0, 0, -1], np.int32)
    return Geometry(2, np.zeros(len(cells) + 1), material, np.arange(len(cells), dtype=np.int32),
                    len(cells), surfaces=np.array(surf), face_off=off, faces=faces)


def csg_module(n_events: int = 1000, seed: int = 7, source_seed: int = 70) -> Workload:
    """Point source at the centre of the quadric-cell module: one primary per event,
    60/20/20 % e-/e+/photon, log-uniform 0.1-10 GeV, isotropic."""
    rng = np.random.default_rng(source_seed)
    n = n_events
    u = rng.random(n)
    species = np.where(u < 0.6, ELECTRON, np.where(u < 0.8, POSITRON, GAMMA)).astype(np.int32)
    energy = _log_uniform(rng, n, 100.0, 10000.0)
    cost = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    sint = np.sqrt(1.0 - cost * cost)
    d = np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)
    ev = Events(np.arange(n, dtype=np.uint32), np.arange(n + 1, dtype=np.int64), species, energy,
                np.zeros((n, 3)), d)
    return Workload("csg_module", [LEAD, LIQUID_ARGON, SILICON, TUNGSTEN],
                    Options(production_cut=0.07), csg_module_geometry(), ev, seed,
                    f"{n} primaries 0.1-10 GeV from the centre of a quadric-cell module")


def barrel_geometry() -> Geometry:
    """Cylinder shells: vacuum core, 5 Si shells of 0.03 cm at r = 4 + 11.5 i,
    vacuum to 150 cm, then 50 Pb/LAr layers of 1 cm pitch (0.2857 Pb + 0.7143 LAr)."""
    b = [0.0]
    mat = []
    for i in range(5):
        r = 4.0 + 11.5 * i
        mat.append(-1)  # vacuum up to r
        b.append(r)
        mat.append(2)  # Si
        b.append(r + 0.03)
    mat.append(-1)
    b.append(150.0)
    pb = 2.0 / 7.0
    for i in range(50):
        r0 = 150.0 + i
        mat.append(0)
        b.append(r0 + pb)
        mat.append(1)
        b.append(r0 + 1.0)
    bounds = np.array(b, np.float64)
    mat = np.array(mat, np.int32)
    n_vol = mat.shape[0]
    # bins: each Si shell its own bin, each calorimeter layer (Pb+LAr) one bin, vacuum -> bin 0
    bins = np.zeros(n_vol, np.int32)
    nb = 1
    for j in range(n_vol):
        if mat[j] == 2:
            bins[j] = nb
            nb += 1
    for j in range(n_vol):
        if mat[j] in (0, 1):
            layer = int(round(bounds[j] - 150.0 - 0.5)) if mat[j] == 1 else int(round(bounds[j] - 150.0))
            bins[j] = nb + layer
    nb += 50
    return Geometry(1, bounds, mat, bins, nb, half_z=300.0, bz=1.0, field_tol=1.0e-5)


def _log_uniform(rng, n, lo, hi):
    return np.exp(np.log(lo) + rng.random(n) * np.log(hi / lo))


def barrel(n_events: int = 1_000_000, seed: int = 4, source_seed: int = 40) -> Workload:
    rng = np.random.default_rng(source_seed)
    n = n_events
    u = rng.random(n)
    species = np.where(u < 0.6, ELECTRON, np.where(u < 0.8, POSITRON, GAMMA)).astype(np.int32)
    energy = _log_uniform(rng, n, 1000.0, 100000.0)
    cmax = np.tanh(1.5)
    cost = -cmax + 2.0 * cmax * rng.random(n)
    phi = 2.0 * np.pi * rng.random(n)
    sint = np.sqrt(1.0 - cost * cost)
    d = np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)
    ev = Events(np.arange(n, dtype=np.uint32), np.arange(n + 1, dtype=np.int64), species,
                energy, np.zeros((n, 3)), d)
    return Workload("barrel", [LEAD, LIQUID_ARGON, SILICON], Options(production_cut=0.07),
                    barrel_geometry(), ev, seed,
                    f"{n} mixed primaries 1-100 GeV, |eta|<1.5, 1 T, cylinders")


def serving(n_events: int = 1000, rate_hz: float = 50.0, seed: int = 5,
            source_seed: int = 50) -> Workload:
    """Poisson arrivals at `rate_hz`; each event U{1..500} primaries of mixed species
    (60% e-, 20% e+, 20% photons), log-uniform 1-100 GeV, normal incidence on the
    calorimeter."""
    rng = np.random.default_rng(source_seed)
    counts = rng.integers(1, 501, size=n_events)
    off = np.zeros(n_events + 1, np.int64)
    off[1:] = np.cumsum(counts)
    n = int(off[-1])
    u = rng.random(n)
    species = np.where(u < 0.6, ELECTRON, np.where(u < 0.8, POSITRON, GAMMA)).astype(np.int32)
    energy = _log_uniform(rng, n, 1000.0, 100000.0)
    arrival = np.cumsum(rng.exponential(1.0 / rate_hz, size=n_events))
    ev = Events(np.arange(n_events, dtype=np.uint32), off, species, energy, np.zeros((n, 3)),
                np.tile(np.array([0.0, 0.0, 1.0]), (n, 1)), arrival)
    return Workload("serving", [LEAD, LIQUID_ARGON], Options(production_cut=0.07),
                    calorimeter_geometry(), ev, seed,
                    f"{n_events} Poisson events at {rate_hz} Hz, 1-500 primaries")


def random_track_states(n: int, n_vol: int, seed: int, e_lo: float = 0.01, e_hi: float = 1.0e5,
                        species: Optional[np.ndarray] = None, vol_material=None,
                        bounds=None, half_xy: float = 20.0, kind: int = 0,
                        half_z: float = 0.0) -> Dict[str, np.ndarray]:
    """Random single-step inputs: species, log-uniform energy, a volume, a point
    inside it (slabs: z between its planes; shells: radius between its radii), an
    isotropic direction, a random key and step count, and interaction lengths left
    (half of them unset).  A quarter of the states sit exactly on the volume's lower
    surface, entering it."""
    rng = np.random.default_rng(seed)
    sp = rng.integers(0, 3, n).astype(np.int32) if species is None else species.astype(np.int32)
    T = _log_uniform(rng, n, e_lo, e_hi)
    vol = rng.integers(0, n_vol, n).astype(np.int32)
    if kind == 1:
        lo, hi = bounds[vol], bounds[vol + 1]
        r = lo + (hi - lo) * rng.random(n)
        on = (rng.random(n) < 0.25) & (lo > 0)
        r = np.where(on, lo, r)
        a = 2.0 * np.pi * rng.random(n)
        pos = np.stack([r * np.cos(a), r * np.sin(a), (2.0 * rng.random(n) - 1.0) * half_z], axis=1)
        cost = 2.0 * rng.random(n) - 1.0
        phi = 2.0 * np.pi * rng.random(n)
        sint = np.sqrt(1.0 - cost * cost)
        d = np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)
        outward = pos[:, 0] * d[:, 0] + pos[:, 1] * d[:, 1] >= 0
        flip = on & ~outward
        d[flip, :2] = -d[flip, :2]
        nlam = np.where(rng.random(n) < 0.5, -1.0, rng.exponential(1.0, n))
        key = rng.integers(0, 2**32, size=(n, 3), dtype=np.uint64).astype(np.uint32)
        nstep = rng.integers(0, 1000, n).astype(np.uint32)
        return dict(species=sp, energy=T, vol=vol, pos=pos, dir=d, nlam=nlam, key=key,
                    nstep=nstep, event=np.arange(n, dtype=np.uint32))
    if bounds is not None:
        lo, hi = bounds[vol], bounds[vol + 1]
        z = lo + (hi - lo) * rng.random(n)
        # a quarter of the states sit exactly on a boundary plane, entering the volume
        on = rng.random(n) < 0.25
        z = np.where(on, lo, z)
    else:
        z = rng.random(n)
    x = (2.0 * rng.random(n) - 1.0) * half_xy
    y = (2.0 * rng.random(n) - 1.0) * half_xy
    cost = 2.0 * rng.random(n) - 1.0
    phi = 2.0 * np.pi * rng.random(n)
    sint = np.sqrt(1.0 - cost * cost)
    d = np.stack([sint * np.cos(phi), sint * np.sin(phi), cost], axis=1)
    if bounds is not None:
        d[:, 2] = np.where(on, np.abs(d[:, 2]), d[:, 2])
    nlam = np.where(rng.random(n) < 0.5, -1.0, rng.exponential(1.0, n))
    key = rng.integers(0, 2**32, size=(n, 3), dtype=np.uint64).astype(np.uint32)
    nstep = rng.integers(0, 1000, n).astype(np.uint32)
    return dict(species=sp, energy=T, vol=vol, pos=np.stack([x, y, z], axis=1), dir=d,
                nlam=nlam, key=key, nstep=nstep, event=np.arange(n, dtype=np.uint32))
