"""MI355X electromagnetic-shower step loop -- Python binding of the C ABI.

Argument marshalling only: every step of the transport runs in the HIP kernels
of ``libemshower.so`` (built in-tree by ``paper_2203_09467_amd/build.py``).
PyTorch provides device memory (the workspace and the primaries' arrays) and
the stream.  If the library is missing this module raises at import time;
there is no CPU fallback.

The functions keep the names of the C entry points (``init_physics_tables``,
``init_geometry``, ``transport_events``, ``tally_read``); ``Context`` bundles
them with the workspace a context needs.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libemshower.so")

if not os.path.exists(LIB_PATH):
    raise ImportError(f"{LIB_PATH} is missing: build it with python -m paper_2203_09467_amd.build")

# One HIP runtime per process: PyTorch loads its own libamdhip64 (SONAME
# libamdhip64.so.7); importing it first makes this library bind to that same
# runtime instead of loading a second copy from /opt/rocm.
import torch  # noqa: E402,F401

_lib = C.CDLL(LIB_PATH)

EMS_OK, EMS_NOT_READY = 0, 1
EMS_FP64, EMS_MIXED = 0, 1
EMS_E_ARG, EMS_E_STATE, EMS_E_CAPACITY, EMS_E_HIP, EMS_E_INTERNAL, EMS_E_STALLED = -1, -2, -3, -4, -5, -6
STATUS = {0: "EMS_OK", 1: "EMS_NOT_READY", -1: "EMS_E_ARG", -2: "EMS_E_STATE",
          -3: "EMS_E_CAPACITY", -4: "EMS_E_HIP", -5: "EMS_E_INTERNAL", -6: "EMS_E_STALLED"}
EMS_FLAG_TIME_STEPS, EMS_FLAG_EVENT_ESCAPE = 1, 2
NGRID = 200


class EmsError(RuntimeError):
    def __init__(self, status: int, where: str):
        msg = _lib.ems_last_error().decode(errors="replace")
        super().__init__(f"{where}: {STATUS.get(status, status)}: {msg}")
        self.status = status


class Config(C.Structure):
    _fields_ = [("pool_capacity", C.c_uint32), ("max_events", C.c_uint32),
                ("max_bins", C.c_uint32), ("queue_capacity", C.c_uint32), ("seed", C.c_uint32),
                ("precision", C.c_int), ("energy_budget", C.c_double), ("flags", C.c_uint32),
                ("iterations_per_sync", C.c_uint32), ("spill_capacity", C.c_uint32),
                ("field_substeps", C.c_uint32)]


class KernelStats(C.Structure):
    _fields_ = [("launches", C.c_uint64), ("tracks_in", C.c_uint64), ("tracks_out", C.c_uint64),
                ("queued", C.c_uint64), ("kernel_ms", C.c_double)]


class Material(C.Structure):
    _fields_ = [("Z", C.c_double), ("A", C.c_double), ("density", C.c_double),
                ("mean_excitation", C.c_double)]


class PhysicsOptions(C.Structure):
    _fields_ = [("tracking_cut", C.c_double), ("production_cut", C.c_double),
                ("compton", C.c_int32), ("photoelectric", C.c_int32), ("pair", C.c_int32),
                ("ionisation", C.c_int32), ("brems", C.c_int32), ("annihilation", C.c_int32),
                ("charged_local", C.c_int32), ("continuous_loss", C.c_int32),
                ("step_alpha", C.c_double), ("step_rfinal", C.c_double),
                ("max_steps", C.c_uint32), ("msc", C.c_int32)]


class Geometry(C.Structure):
    _fields_ = [("kind", C.c_int32), ("n_vol", C.c_int32), ("bounds", C.POINTER(C.c_double)),
                ("material", C.POINTER(C.c_int32)), ("tally_bin", C.POINTER(C.c_int32)),
                ("n_bins", C.c_int32), ("half_x", C.c_double), ("half_y", C.c_double),
                ("half_z", C.c_double), ("bz", C.c_double), ("field_tol", C.c_double),
                ("n_surf", C.c_int32), ("surfaces", C.POINTER(C.c_double)),
                ("face_off", C.POINTER(C.c_int32)), ("faces", C.POINTER(C.c_int32))]


class EventBatch(C.Structure):
    _fields_ = [("n_events", C.c_uint32), ("event_ids", C.POINTER(C.c_uint32)),
                ("offsets", C.POINTER(C.c_int64)), ("species", C.c_void_p),
                ("energy", C.c_void_p), ("pos", C.c_void_p), ("dir", C.c_void_p)]


class Progress(C.Structure):
    _fields_ = [("alive", C.c_uint64), ("queued_primaries", C.c_uint64),
                ("queued_events", C.c_uint64), ("iterations", C.c_uint64),
                ("track_steps", C.c_uint64), ("deferred", C.c_uint64),
                ("peak_alive", C.c_uint64), ("spilled", C.c_uint64),
                ("spilled_total", C.c_uint64), ("events_done", C.c_uint64)]


class IterationRecord(C.Structure):
    _fields_ = [("photons", C.c_uint32), ("charged", C.c_uint32), ("interactions", C.c_uint32),
                ("tracks_out", C.c_uint32), ("waiting_primaries", C.c_uint64),
                ("spilled", C.c_uint64), ("ms", C.c_double)]


ITERATION_DTYPE = np.dtype([("photons", "u4"), ("charged", "u4"), ("interactions", "u4"),
                            ("tracks_out", "u4"), ("waiting_primaries", "u8"), ("spilled", "u8"),
                            ("ms", "f8")])


class StepRecord(C.Structure):
    _fields_ = [("dep", C.c_double), ("esc", C.c_double), ("killed", C.c_double),
                ("step_len", C.c_double), ("limiter", C.c_int32), ("process", C.c_int32),
                ("n_pair", C.c_int32), ("n_annih", C.c_int32), ("n_out", C.c_int32),
                ("escaped", C.c_int32)]


SOA_FIELDS = [("x", "f8"), ("y", "f8"), ("z", "f8"), ("u", "f8"), ("v", "f8"), ("w", "f8"),
              ("T", "f8"), ("nlam", "f8"), ("k0", "u4"), ("k1", "u4"), ("k2", "u4"),
              ("event", "u4"), ("nstep", "u4"), ("species", "i4"), ("vol", "i4"), ("vcap", "u4")]


class TrackSoA(C.Structure):
    _fields_ = [(n, C.c_void_p) for n, _ in SOA_FIELDS]


RECORD_DTYPE = np.dtype([("dep", "f8"), ("esc", "f8"), ("killed", "f8"), ("step_len", "f8"),
                         ("limiter", "i4"), ("process", "i4"), ("n_pair", "i4"),
                         ("n_annih", "i4"), ("n_out", "i4"), ("escaped", "i4")])
assert RECORD_DTYPE.itemsize == C.sizeof(StepRecord)
assert ITERATION_DTYPE.itemsize == C.sizeof(IterationRecord)

_P = C.POINTER
_sigs = {
    "ems_workspace_bytes": (C.c_size_t, [_P(Config)]),
    "ems_create": (C.c_int, [_P(Config), C.c_void_p, C.c_size_t, _P(C.c_void_p)]),
    "ems_create_static": (C.c_int, [_P(Config), _P(C.c_void_p)]),
    "ems_destroy": (None, [C.c_void_p]),
    "ems_last_error": (C.c_char_p, []),
    "init_physics_tables": (C.c_int, [C.c_void_p, _P(Material), C.c_int32, _P(PhysicsOptions),
                                      C.c_void_p]),
    "init_geometry": (C.c_int, [C.c_void_p, _P(Geometry), C.c_void_p]),
    "transport_events": (C.c_int, [C.c_void_p, _P(EventBatch), C.c_int32, C.c_void_p,
                                   _P(Progress)]),
    "tally_read": (C.c_int, [C.c_void_p, C.c_uint32, _P(C.c_uint32), _P(C.c_double),
                             _P(C.c_double), _P(C.c_uint64), _P(C.c_uint64), _P(C.c_int32),
                             C.c_void_p]),
    "ems_run_counters": (C.c_int, [C.c_void_p, _P(C.c_uint64), _P(C.c_uint64), _P(C.c_uint64),
                                   C.c_void_p]),
    "ems_step_stats": (C.c_int, [C.c_void_p, _P(KernelStats), C.c_int32]),
    "ems_iteration_log": (C.c_int, [C.c_void_p, C.c_void_p, C.c_uint64, _P(C.c_uint64), C.c_int32]),
    "ems_step_once": (C.c_int, [C.c_void_p, _P(TrackSoA), C.c_uint32, C.c_void_p, _P(TrackSoA),
                                _P(C.c_uint32), C.c_void_p]),
}
for _name, (_res, _args) in _sigs.items():
    _f = getattr(_lib, _name)
    _f.restype = _res
    _f.argtypes = _args

EXPORTED = list(_sigs)


def _check(st: int, where: str, ok=(EMS_OK,)):
    if st not in ok:
        raise EmsError(st, where)
    return st


def _stream(stream=None):
    import torch
    s = stream if stream is not None else torch.cuda.current_stream()
    return C.c_void_p(s.cuda_stream)


def _np_ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(C.POINTER(ct))


# --------------------------------------------------------------------------- raw entry points
def workspace_bytes(cfg: Config) -> int:
    return int(_lib.ems_workspace_bytes(C.byref(cfg)))


def create(cfg: Config, workspace_ptr: int, nbytes: int) -> C.c_void_p:
    h = C.c_void_p()
    _check(_lib.ems_create(C.byref(cfg), C.c_void_p(workspace_ptr), nbytes, C.byref(h)), "ems_create")
    return h


def create_static(cfg: Config) -> C.c_void_p:
    """A context over the library's static device scratch (no allocation)."""
    h = C.c_void_p()
    _check(_lib.ems_create_static(C.byref(cfg), C.byref(h)), "ems_create_static")
    return h


def init_physics_tables(ctx, materials, options, stream=None):
    mats = (Material * len(materials))(*[Material(*m) for m in materials])
    o = PhysicsOptions()
    for f, _ in PhysicsOptions._fields_:
        setattr(o, f, getattr(options, f))
    _check(_lib.init_physics_tables(ctx, mats, len(materials), C.byref(o), _stream(stream)),
           "init_physics_tables")


def init_geometry(ctx, geometry, stream=None):
    b = np.ascontiguousarray(geometry.bounds, np.float64)
    m = np.ascontiguousarray(geometry.material, np.int32)
    t = np.ascontiguousarray(geometry.tally_bin, np.int32)
    g = Geometry(int(geometry.kind), int(m.shape[0]), _np_ptr(b, C.c_double), _np_ptr(m, C.c_int32),
                 _np_ptr(t, C.c_int32), int(geometry.n_bins), float(geometry.half_x),
                 float(geometry.half_y), float(geometry.half_z), float(geometry.bz),
                 float(geometry.field_tol))
    keep = []
    if getattr(geometry, "surfaces", None) is not None:
        sf = np.ascontiguousarray(geometry.surfaces, np.float64).reshape(-1)
        fo = np.ascontiguousarray(geometry.face_off, np.int32)
        fc = np.ascontiguousarray(geometry.faces, np.int32)
        keep = [sf, fo, fc]
        g.n_surf = sf.shape[0] // 10
        g.surfaces = _np_ptr(sf, C.c_double)
        g.face_off = _np_ptr(fo, C.c_int32)
        g.faces = _np_ptr(fc, C.c_int32)
    _check(_lib.init_geometry(ctx, C.byref(g), _stream(stream)), "init_geometry")
    del keep


def transport_events(ctx, batch: Optional["DeviceEvents"], max_iterations: int = -1,
                     stream=None) -> Progress:
    pr = Progress()
    if batch is None:
        bp = None
    else:
        bp = C.byref(batch.c_struct())
    _check(_lib.transport_events(ctx, bp, int(max_iterations), _stream(stream), C.byref(pr)),
           "transport_events")
    return pr


def tally_read(ctx, event_ids, n_bins: int, stream=None, steps: bool = False,
               escape: bool = False):
    """Returns (dep, ledger, status), followed by the per-event track-steps by species
    (n x 3) if `steps` and the per-event escape spectra (n x 3 x 200) if `escape`."""
    ids = np.ascontiguousarray(event_ids, np.uint32)
    n = ids.shape[0]
    dep = np.zeros((n, n_bins), np.float64)
    ledger = np.zeros((n, 5), np.float64)
    status = np.zeros(n, np.int32)
    st = np.zeros((n, 3), np.uint64) if steps else None
    esc = np.zeros((n, 3, NGRID), np.uint64) if escape else None
    _check(_lib.tally_read(ctx, n, _np_ptr(ids, C.c_uint32), _np_ptr(dep, C.c_double),
                           _np_ptr(ledger, C.c_double),
                           None if st is None else _np_ptr(st, C.c_uint64),
                           None if esc is None else _np_ptr(esc, C.c_uint64),
                           _np_ptr(status, C.c_int32), _stream(stream)),
           "tally_read", ok=(EMS_OK, EMS_NOT_READY))
    out = (dep, ledger, status)
    if steps:
        out += (st,)
    if escape:
        out += (esc,)
    return out


LIFE_BINS = 17


def run_counters(ctx, stream=None, life=False):
    """(steps by species, escape histogram 3 x 200[, steps-per-track histogram 3 x 17])."""
    steps = np.zeros(3, np.uint64)
    hist = np.zeros((3, NGRID), np.uint64)
    lh = np.zeros((3, LIFE_BINS), np.uint64)
    _check(_lib.ems_run_counters(ctx, _np_ptr(steps, C.c_uint64), _np_ptr(hist, C.c_uint64),
                                 _np_ptr(lh, C.c_uint64), _stream(stream)), "ems_run_counters")
    return (steps, hist, lh) if life else (steps, hist)


# --------------------------------------------------------------------------- torch-side helpers
class DeviceEvents:
    """Primaries of a workloads.Events batch, resident on the GPU."""

    def __init__(self, events, device="cuda"):
        import torch
        self.ids = np.ascontiguousarray(events.event_ids, np.uint32)
        self.offsets = np.ascontiguousarray(events.offsets, np.int64)
        self.species = torch.as_tensor(np.ascontiguousarray(events.species, np.int32), device=device)
        self.energy = torch.as_tensor(np.ascontiguousarray(events.energy, np.float64), device=device)
        self.pos = torch.as_tensor(np.ascontiguousarray(events.pos, np.float64), device=device)
        self.dir = torch.as_tensor(np.ascontiguousarray(events.dir, np.float64), device=device)

    @property
    def n_events(self):
        return int(self.ids.shape[0])

    def c_struct(self) -> EventBatch:
        self._keep = (self.ids, self.offsets)
        return EventBatch(self.n_events, _np_ptr(self.ids, C.c_uint32), _np_ptr(self.offsets, C.c_int64),
                          self.species.data_ptr(), self.energy.data_ptr(), self.pos.data_ptr(),
                          self.dir.data_ptr())

    def slice(self, a: int, b: int) -> "EventSlice":
        """Events [a, b) of this batch, without copying the device arrays."""
        return EventSlice(self, a, b)


class EventSlice:
    """A contiguous run of events of a DeviceEvents batch (views of its arrays)."""

    def __init__(self, parent: DeviceEvents, a: int, b: int):
        self.parent = parent
        self.ids = np.ascontiguousarray(parent.ids[a:b])
        r0 = int(parent.offsets[a])
        self.offsets = np.ascontiguousarray(parent.offsets[a:b + 1] - r0)
        self.r0 = r0

    @property
    def n_events(self):
        return int(self.ids.shape[0])

    def c_struct(self) -> EventBatch:
        p, r0 = self.parent, self.r0
        self._keep = (self.ids, self.offsets)
        return EventBatch(self.n_events, _np_ptr(self.ids, C.c_uint32), _np_ptr(self.offsets, C.c_int64),
                          p.species.data_ptr() + 4 * r0, p.energy.data_ptr() + 8 * r0,
                          p.pos.data_ptr() + 24 * r0, p.dir.data_ptr() + 24 * r0)


class Context:
    """A transport context over a torch-allocated workspace."""

    def __init__(self, pool_capacity=1 << 20, max_events=1024, max_bins=128,
                 queue_capacity=1 << 20, seed=1, precision=EMS_FP64, energy_budget=0.0,
                 time_steps=False, iterations_per_sync=0, event_escape=False, spill_capacity=0,
                 field_substeps=0, device="cuda"):
        import torch
        flags = (EMS_FLAG_TIME_STEPS if time_steps else 0) | (EMS_FLAG_EVENT_ESCAPE if event_escape else 0)
        self.cfg = Config(pool_capacity, max_events, max_bins, queue_capacity, seed, precision,
                          energy_budget, flags, iterations_per_sync, spill_capacity, field_substeps)
        nbytes = workspace_bytes(self.cfg)
        if nbytes == 0:
            raise EmsError(-1, "ems_workspace_bytes")
        self.workspace = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        self.h = create(self.cfg, aligned, nbytes)
        self.n_bins = None

    def close(self):
        if getattr(self, "h", None):
            _lib.ems_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def setup(self, materials, options, geometry, stream=None):
        init_physics_tables(self.h, materials, options, stream)
        init_geometry(self.h, geometry, stream)
        self.n_bins = int(geometry.n_bins)

    def transport(self, batch=None, max_iterations=-1, stream=None) -> Progress:
        return transport_events(self.h, batch, max_iterations, stream)

    def read(self, event_ids, stream=None, steps=False, escape=False):
        return tally_read(self.h, event_ids, self.n_bins, stream, steps, escape)

    def counters(self, stream=None, life=False):
        return run_counters(self.h, stream, life)

    def iteration_log(self, reset=False) -> np.ndarray:
        """Per-iteration records (numpy structured array, ITERATION_DTYPE)."""
        n = C.c_uint64()
        _check(_lib.ems_iteration_log(self.h, None, 0, C.byref(n), 0), "ems_iteration_log")
        out = np.zeros(n.value, ITERATION_DTYPE)
        _check(_lib.ems_iteration_log(self.h, C.c_void_p(out.ctypes.data), n.value, C.byref(n),
                                      1 if reset else 0), "ems_iteration_log")
        return out[:n.value]

    def step_stats(self, reset=False) -> KernelStats:
        st = KernelStats()
        _check(_lib.ems_step_stats(self.h, C.byref(st), 1 if reset else 0), "ems_step_stats")
        return st

    def step_once(self, states: dict, stream=None):
        """Step the given states (dict of numpy arrays: species, energy, vol, pos, dir, nlam,
        key, nstep, event, optionally vcap) once; returns (records, outputs dict of numpy
        arrays)."""
        import torch
        n = len(states["species"])
        cols = {
            "x": states["pos"][:, 0], "y": states["pos"][:, 1], "z": states["pos"][:, 2],
            "u": states["dir"][:, 0], "v": states["dir"][:, 1], "w": states["dir"][:, 2],
            "T": states["energy"], "nlam": states["nlam"], "k0": states["key"][:, 0],
            "k1": states["key"][:, 1], "k2": states["key"][:, 2], "event": states["event"],
            "nstep": states["nstep"], "species": states["species"], "vol": states["vol"],
            "vcap": states.get("vcap", np.zeros(n, np.uint32)),
        }
        dev_in = {}
        for k, dt in SOA_FIELDS:
            a = np.ascontiguousarray(cols[k], dt)
            dev_in[k] = torch.as_tensor(a.view(np.int32) if dt == "u4" else a, device="cuda")
        dev_out = {k: torch.empty(3 * n, dtype=getattr(torch, {"f8": "float64", "u4": "int32",
                                                             "i4": "int32"}[dt]), device="cuda")
                   for k, dt in SOA_FIELDS}
        rec = torch.empty(n * RECORD_DTYPE.itemsize, dtype=torch.uint8, device="cuda")
        sin = TrackSoA(*[dev_in[k].data_ptr() for k, _ in SOA_FIELDS])
        sout = TrackSoA(*[dev_out[k].data_ptr() for k, _ in SOA_FIELDS])
        n_out = C.c_uint32()
        _check(_lib.ems_step_once(self.h, C.byref(sin), n, C.c_void_p(rec.data_ptr()), C.byref(sout),
                                  C.byref(n_out), _stream(stream)), "ems_step_once")
        records = np.frombuffer(rec.cpu().numpy().tobytes(), dtype=RECORD_DTYPE)
        m = n_out.value
        out = {}
        for k, dt in SOA_FIELDS:
            a = dev_out[k][:m].cpu().numpy()
            out[k] = a.view(np.uint32) if dt == "u4" else a
        return records, out
