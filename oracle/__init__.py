"""ctypes binding of the CPU oracle -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of
``bench.py`` may import this package.  It wraps ``liboracle.so`` (built by
``oracle/build.py`` from the plain C sources next to it) and shares no code
with the product package.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Dict

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "liboracle.so")

GAMMA, ELECTRON, POSITRON = 0, 1, 2
NGRID = 200
LIFE_BINS = 17


class Material(C.Structure):
    _fields_ = [("Z", C.c_double), ("A", C.c_double), ("density", C.c_double),
                ("mean_excitation", C.c_double)]


class Options(C.Structure):
    _fields_ = [("tracking_cut", C.c_double), ("production_cut", C.c_double),
                ("compton", C.c_int), ("photoelectric", C.c_int), ("pair", C.c_int),
                ("ionisation", C.c_int), ("brems", C.c_int), ("annihilation", C.c_int),
                ("charged_local", C.c_int), ("continuous_loss", C.c_int),
                ("step_alpha", C.c_double), ("step_rfinal", C.c_double),
                ("max_steps", C.c_uint32), ("msc", C.c_int)]


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int), ("n_vol", C.c_int), ("bounds", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_int)), ("tally_bin", C.POINTER(C.c_int)),
                ("n_bins", C.c_int), ("half_x", C.c_double), ("half_y", C.c_double),
                ("half_z", C.c_double), ("bz", C.c_double), ("field_tol", C.c_double),
                ("n_surf", C.c_int), ("surf", C.POINTER(C.c_double)),
                ("face_off", C.POINTER(C.c_int)), ("faces", C.POINTER(C.c_int))]


class Track(C.Structure):
    _fields_ = [("species", C.c_int), ("x", C.c_double), ("y", C.c_double), ("z", C.c_double),
                ("u", C.c_double), ("v", C.c_double), ("w", C.c_double), ("T", C.c_double),
                ("nlam", C.c_double), ("key", C.c_uint32 * 3), ("event", C.c_uint32),
                ("nstep", C.c_uint32), ("vol", C.c_int), ("vac_caps", C.c_uint32)]


class StepResult(C.Structure):
    _fields_ = [("out", Track * 3), ("n_out", C.c_int), ("parent_alive", C.c_int),
                ("dep", C.c_double), ("dep_bin", C.c_int), ("esc", C.c_double),
                ("esc_species", C.c_int), ("escaped", C.c_int), ("killed", C.c_double),
                ("n_pair", C.c_int), ("n_annih", C.c_int), ("limiter", C.c_int),
                ("process", C.c_int), ("step_len", C.c_double)]


_lib = None


def lib() -> C.CDLL:
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            from . import build as _b
            _b.build()
        L = C.CDLL(LIB_PATH)
        d, u32, i = C.c_double, C.c_uint32, C.c_int
        P = C.POINTER
        for name in ["or_kn_sigma"]:
            getattr(L, name).restype = d
        sigs = {
            "or_kn_sigma": (d, [d]), "or_kn_dsigma": (d, [d, d]), "or_pe_sigma": (d, [d, d]),
            "or_pair_Sigma": (d, [d, d]), "or_pair_dSigma": (d, [d, d, d]),
            "or_brems_Sigma": (d, [d, d, d]), "or_brems_dSigma": (d, [d, d, d]),
            "or_brems_Srad": (d, [d, d, d]), "or_moller_sigma": (d, [d, d]),
            "or_moller_dsigma": (d, [d, d]), "or_bhabha_sigma": (d, [d, d]),
            "or_bhabha_dsigma": (d, [d, d]), "or_heitler_sigma": (d, [d, d]),
            "or_heitler_dsigma": (d, [d, d, d]), "or_scol": (d, [i, d, d, d, d]),
            "or_radiation_length": (d, [d, d, d]), "or_msc_theta0": (d, [d, d, d]),
            "or_accept_moller": (d, [d, d]), "or_accept_bhabha": (d, [d, d]),
            "or_accept_heitler": (d, [d, d]), "or_accept_kn": (d, [d, d]),
            "or_sample_kn": (i, [d, P(d), i, P(d), P(d)]),
            "or_sample_pair": (i, [d, P(d), i, P(d)]),
            "or_sample_brems": (i, [d, d, P(d), i, P(d)]),
            "or_sample_moller": (i, [d, d, P(d), i, P(d)]),
            "or_sample_bhabha": (i, [d, d, P(d), i, P(d)]),
            "or_sample_heitler": (i, [d, P(d), i, P(d)]),
            "or_philox4x32_10": (None, [P(u32), P(u32), P(u32)]),
            "or_uniform": (d, [u32, P(u32), u32, u32]),
            "or_primary_key": (None, [u32, u32, u32, P(u32)]),
            "or_child_key": (None, [u32, P(u32), u32, u32, P(u32)]),
            "or_create": (C.c_void_p, [P(Material), i, P(Options), P(Geometry)]),
            "or_destroy": (None, [C.c_void_p]),
            "or_grid_energy": (d, [C.c_void_p, i]),
            "or_table_node": (d, [C.c_void_p, i, i, i, i]),
            "or_table_interp": (d, [C.c_void_p, i, i, i, d]),
            "or_range_inverse": (d, [C.c_void_p, i, i, d]),
            "or_cut_electron": (d, [C.c_void_p, i]), "or_cut_gamma": (d, [C.c_void_p, i]),
            "or_range_at_cut": (d, [C.c_void_p, i, i]),
            "or_material_X0": (d, [C.c_void_p, i]),
            "or_locate": (i, [C.c_void_p, d, d, d, d, d, d]),
            "or_distance": (d, [C.c_void_p, i, P(d), P(d), P(i)]),
            "or_step": (i, [C.c_void_p, u32, P(Track), P(StepResult)]),
            "or_rotate": (None, [P(d), d, d, P(d)]),
            "or_csg_side": (i, [P(d), P(d), P(d)]),
            "or_csg_exit": (d, [P(d), P(d), P(d), i]),
            "or_field_kappa": (d, [d, d, d]),
            "or_rk4": (None, [d, d, P(d), P(d), P(d), P(d)]),
            "or_field_move": (i, [C.c_void_p, i, d, d, i, P(d), P(d), P(d), P(i)]),
            "or_run_batch": (i, [C.c_void_p, u32, i, P(u32), P(C.c_int64), P(i), P(d), P(d),
                                 P(d), P(d), P(d), P(C.c_int64), P(C.c_int64), C.c_void_p,
                                 C.c_void_p]),
            "or_life_bin": (i, [C.c_long]),
        }
        for name, (res, args) in sigs.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# ---------------------------------------------------------------- RNG
def philox(ctr, key):
    c = (C.c_uint32 * 4)(*[int(x) & 0xFFFFFFFF for x in ctr])
    k = (C.c_uint32 * 2)(*[int(x) & 0xFFFFFFFF for x in key])
    o = (C.c_uint32 * 4)()
    lib().or_philox4x32_10(c, k, o)
    return [int(x) for x in o]


def uniform(seed, key, step, draw):
    k = (C.c_uint32 * 3)(*[int(x) for x in key])
    return lib().or_uniform(seed, k, step, draw)


def primary_key(seed, event_id, index):
    o = (C.c_uint32 * 3)()
    lib().or_primary_key(seed, event_id, index, o)
    return [int(x) for x in o]


def child_key(seed, parent, step, ordinal):
    p = (C.c_uint32 * 3)(*[int(x) for x in parent])
    o = (C.c_uint32 * 3)()
    lib().or_child_key(seed, p, step, ordinal, o)
    return [int(x) for x in o]


# ---------------------------------------------------------------- samplers
def sample(name: str, params, u: np.ndarray):
    """Run one array-fed sampler; returns (value(s), draws consumed)."""
    L = lib()
    u = np.ascontiguousarray(u, np.float64)
    a = C.c_double()
    b = C.c_double()
    pu = _ptr(u, C.c_double)
    if name == "kn":
        n = L.or_sample_kn(params[0], pu, len(u), C.byref(a), C.byref(b))
        return (a.value, b.value), n
    fn = {"pair": L.or_sample_pair, "heitler": L.or_sample_heitler}.get(name)
    if fn is not None:
        n = fn(params[0], pu, len(u), C.byref(a))
        return a.value, n
    fn = {"brems": L.or_sample_brems, "moller": L.or_sample_moller,
          "bhabha": L.or_sample_bhabha}[name]
    n = fn(params[0], params[1], pu, len(u), C.byref(a))
    return a.value, n


# ---------------------------------------------------------------- world
def _options(opts) -> Options:
    o = Options()
    for f, _ in Options._fields_:
        setattr(o, f, getattr(opts, f))
    return o


class World:
    """Materials + tables + geometry + options, built by the oracle from the inputs."""

    def __init__(self, materials, options, geometry):
        L = lib()
        mats = (Material * max(1, len(materials)))()
        for i, m in enumerate(materials):
            mats[i] = Material(*m)
        self._bounds = np.ascontiguousarray(geometry.bounds, np.float64)
        self._mat = np.ascontiguousarray(geometry.material, np.int32)
        self._bin = np.ascontiguousarray(geometry.tally_bin, np.int32)
        g = Geometry(int(geometry.kind), int(self._mat.shape[0]), _ptr(self._bounds, C.c_double),
                     _ptr(self._mat, C.c_int), _ptr(self._bin, C.c_int), int(geometry.n_bins),
                     float(geometry.half_x), float(geometry.half_y), float(geometry.half_z),
                     float(geometry.bz), float(geometry.field_tol))
        if getattr(geometry, "surfaces", None) is not None:
            self._surf = np.ascontiguousarray(geometry.surfaces, np.float64).reshape(-1)
            self._foff = np.ascontiguousarray(geometry.face_off, np.int32)
            self._faces = np.ascontiguousarray(geometry.faces, np.int32)
            g.n_surf = self._surf.shape[0] // 10
            g.surf = _ptr(self._surf, C.c_double)
            g.face_off = _ptr(self._foff, C.c_int)
            g.faces = _ptr(self._faces, C.c_int)
        self.options = options
        self.geometry = geometry
        self.n_bins = int(geometry.n_bins)
        o = _options(options)
        self.h = L.or_create(mats, len(materials), C.byref(o), C.byref(g))
        if not self.h:
            raise ValueError("oracle: invalid world description")

    def __del__(self):
        h = getattr(self, "h", None)
        if h and _lib is not None:
            _lib.or_destroy(h)
            self.h = None

    # tables -------------------------------------------------------------
    def grid_energy(self, i):
        return lib().or_grid_energy(self.h, i)

    def node(self, mat, species, q, i):
        return lib().or_table_node(self.h, mat, species, q, i)

    def interp(self, mat, species, q, T):
        return lib().or_table_interp(self.h, mat, species, q, T)

    def range_inverse(self, mat, species, r):
        return lib().or_range_inverse(self.h, mat, species, r)

    def cut_electron(self, mat):
        return lib().or_cut_electron(self.h, mat)

    def cut_gamma(self, mat):
        return lib().or_cut_gamma(self.h, mat)

    def range_at_cut(self, mat, species):
        return lib().or_range_at_cut(self.h, mat, species)

    def X0(self, mat):
        return lib().or_material_X0(self.h, mat)

    def locate(self, pos, d):
        return lib().or_locate(self.h, *[float(x) for x in pos], *[float(x) for x in d])

    def field_move(self, vol, kappa, s_max, vacuum, pos, d):
        """Curved move of a charged track; returns (status, path, pos, dir, next)."""
        p = (C.c_double * 3)(*pos)
        q = (C.c_double * 3)(*d)
        sl = C.c_double()
        nx = C.c_int()
        st = lib().or_field_move(self.h, vol, kappa, s_max, vacuum, p, q, C.byref(sl), C.byref(nx))
        return st, sl.value, list(p), list(q), nx.value

    def distance(self, vol, pos, d):
        p = (C.c_double * 3)(*pos)
        q = (C.c_double * 3)(*d)
        nx = C.c_int()
        s = lib().or_distance(self.h, vol, p, q, C.byref(nx))
        return s, nx.value

    # transport ----------------------------------------------------------
    def step_tracks(self, seed: int, st: Dict[str, np.ndarray]):
        """Step every state in `st` (dict of arrays as made by
        workloads.random_track_states) once; returns a list of StepResult copies."""
        L = lib()
        n = len(st["species"])
        out = []
        r = StepResult()
        t = Track()
        for i in range(n):
            t.species = int(st["species"][i])
            t.x, t.y, t.z = (float(v) for v in st["pos"][i])
            t.u, t.v, t.w = (float(v) for v in st["dir"][i])
            t.T = float(st["energy"][i])
            t.nlam = float(st["nlam"][i])
            for j in range(3):
                t.key[j] = int(st["key"][i][j])
            t.event = int(st["event"][i])
            t.nstep = int(st["nstep"][i])
            t.vol = int(st["vol"][i])
            t.vac_caps = int(st["vcap"][i]) if "vcap" in st else 0
            if L.or_step(self.h, seed, C.byref(t), C.byref(r)) != 0:
                raise RuntimeError("oracle step failed")
            c = StepResult()
            C.pointer(c)[0] = r
            out.append(c)
        return out

    def run_events(self, seed: int, ev, esc_hist: bool = False, life_hist: bool = False):
        """Transport a workloads.Events batch; returns dict with dep (n_events x n_bins),
        ledger (n_events x 5: e_in, escaped, killed, n_pair, n_annih), steps[3], tracks[3]
        and optionally the escape histogram (3 x 200) and the steps-per-track
        histogram (3 x LIFE_BINS)."""
        L = lib()
        ne = ev.n_events
        dep = np.zeros((ne, self.n_bins), np.float64)
        ledger = np.zeros((ne, 5), np.float64)
        steps = np.zeros(3, np.int64)
        tracks = np.zeros(3, np.int64)
        hist = np.zeros((3, NGRID), np.float64) if esc_hist else None
        lh = np.zeros((3, LIFE_BINS), np.float64) if life_hist else None
        ids = np.ascontiguousarray(ev.event_ids, np.uint32)
        off = np.ascontiguousarray(ev.offsets, np.int64)
        sp = np.ascontiguousarray(ev.species, np.int32)
        T = np.ascontiguousarray(ev.energy, np.float64)
        pos = np.ascontiguousarray(ev.pos, np.float64)
        d = np.ascontiguousarray(ev.dir, np.float64)
        rc = L.or_run_batch(self.h, seed, ne, _ptr(ids, C.c_uint32), _ptr(off, C.c_int64),
                            _ptr(sp, C.c_int), _ptr(T, C.c_double), _ptr(pos, C.c_double),
                            _ptr(d, C.c_double), _ptr(dep, C.c_double), _ptr(ledger, C.c_double),
                            _ptr(steps, C.c_int64), _ptr(tracks, C.c_int64),
                            None if hist is None else hist.ctypes.data,
                            None if lh is None else lh.ctypes.data)
        if rc != 0:
            raise RuntimeError("oracle transport failed")
        res = dict(dep=dep, ledger=ledger, steps=steps, tracks=tracks)
        if hist is not None:
            res["esc_hist"] = hist
        if lh is not None:
            res["life_hist"] = lh
        return res


def csg_side(q, p, d) -> int:
    """Side (+1 / -1) of quadric surface q (10 coefficients) at p moving along d."""
    a = lambda v: (C.c_double * len(v))(*[float(x) for x in v])
    return lib().or_csg_side(a(q), a(p), a(d))


def csg_exit(q, p, d, sigma: int) -> float:
    """Distance along d from p to where quadric q leaves side sigma (inf: never)."""
    a = lambda v: (C.c_double * len(v))(*[float(x) for x in v])
    return lib().or_csg_exit(a(q), a(p), a(d), int(sigma))


def rotate(d, c, phi):
    """The oracle's rotation of unit vector d by polar cosine c and azimuth phi."""
    a = (C.c_double * 3)(*[float(x) for x in d])
    o = (C.c_double * 3)()
    lib().or_rotate(a, float(c), float(phi), o)
    return np.array(list(o))


def closed(name: str, *args) -> float:
    return getattr(lib(), "or_" + name)(*args)
