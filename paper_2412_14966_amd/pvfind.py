"""Python binding of libpvfind (include/pvfind.h) over ctypes.

Argument marshalling only: every step of the path runs in the library's HIP
kernels.  PyTorch provides device memory and streams.  If the built library
is missing, loading fails with an error instead of falling back to anything.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
from typing import Dict, Optional

import numpy as np

from . import synth

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libpvfind.so")

PV_OK, PV_EINVAL, PV_EHIP, PV_ENOMEM, PV_EBUSY = 0, -1, -2, -3, -4
PV_EV_NONFINITE_INPUT, PV_EV_TOO_MANY_TRACKS, PV_EV_VERTEX_OVERFLOW, PV_EV_OFFSETS_INVALID = 1, 2, 4, 8
PV_EV_FIT_FAILED = 16
PV_VX_NOT_CONVERGED, PV_VX_FP64_INVERSION = 1, 2


class PvError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"libpvfind error {code}: {msg}")
        self.code = code


class pv_tracks(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "y", "z", "tx", "ty", "cov_xx", "cov_xtx", "cov_txtx")]


class pv_beamline(ctypes.Structure):
    _fields_ = [("x", ctypes.c_float), ("y", ctypes.c_float), ("tx", ctypes.c_float), ("ty", ctypes.c_float)]


class pv_params(ctypes.Structure):
    _fields_ = [
        ("z_min", ctypes.c_float), ("z_max", ctypes.c_float), ("dz", ctypes.c_float), ("z_gas", ctypes.c_float),
        ("sigma_max_pp", ctypes.c_float), ("sigma_max_gas", ctypes.c_float), ("u0", ctypes.c_float),
        ("frac_bits", ctypes.c_int32), ("proto_thr", ctypes.c_int32), ("dip_prom", ctypes.c_int32),
        ("min_int_pp", ctypes.c_int32), ("min_int_gas", ctypes.c_int32),
        ("part_min_pp", ctypes.c_int32), ("part_min_gas", ctypes.c_int32),
        ("pv_min_pp", ctypes.c_int32), ("pv_min_gas", ctypes.c_int32), ("max_iter", ctypes.c_int32),
        ("chi2_max", ctypes.c_float), ("conv_dchi2", ctypes.c_float), ("conv_dz", ctypes.c_float),
        ("max_rho_pp", ctypes.c_float), ("cond_fp64", ctypes.c_float), ("sing_ratio", ctypes.c_float),
        ("max_tracks_per_event", ctypes.c_int32), ("max_vertices_per_event", ctypes.c_int32),
        ("assoc_mode", ctypes.c_int32), ("chi2_max_mv", ctypes.c_float), ("chi2_window_mv", ctypes.c_float),
        ("conv_dz_mv", ctypes.c_float), ("dup_ratio", ctypes.c_float), ("w_count_mv", ctypes.c_float),
        ("peak_mode", ctypes.c_int32),
    ]


class pv_vertices_out(ctypes.Structure):
    _fields_ = [("vertices", ctypes.c_void_p), ("n_vertices", ctypes.c_void_p), ("status", ctypes.c_void_p)]


class pv_track_out(ctypes.Structure):
    _fields_ = [("vertex", ctypes.c_void_p), ("weight", ctypes.c_void_p)]


class pv_debug_out(ctypes.Structure):
    _fields_ = [("hist", ctypes.c_void_p), ("clusters", ctypes.c_void_p), ("n_clusters", ctypes.c_void_p),
                ("zpoca", ctypes.c_void_p), ("sigma", ctypes.c_void_p), ("bin", ctypes.c_void_p),
                ("stage_cycles", ctypes.c_void_p)]


class pv_schedule(ctypes.Structure):
    _fields_ = [("waves_per_team", ctypes.c_int32), ("track_capacity", ctypes.c_int32),
                ("persistent", ctypes.c_int32), ("teams_per_cu", ctypes.c_int32)]


# 64-byte vertex record and 32-byte cluster record, as numpy dtypes
VERTEX_DTYPE = np.dtype([("x", "<f4"), ("y", "<f4"), ("z", "<f4"), ("cov", "<f4", (6,)), ("chi2", "<f4"),
                         ("ndof", "<f4"), ("z_seed", "<f4"), ("n_tracks", "<i4"), ("bin_lo", "<i2"),
                         ("bin_hi", "<i2"), ("peak_bin", "<i2"), ("n_iter", "u1"), ("flags", "u1"),
                         ("reserved", "<i4")])
CLUSTER_DTYPE = np.dtype([("lo", "<i4"), ("hi", "<i4"), ("peak", "<i4"), ("z_seed", "<f4"), ("kept", "<i4"),
                          ("n_assoc", "<i4"), ("own_lo", "<i4"), ("own_hi", "<i4")])
assert VERTEX_DTYPE.itemsize == 64 and CLUSTER_DTYPE.itemsize == 32

_lib = None


def lib():
    """Load libpvfind.so (built by ``python -m paper_2412_14966_amd.build``)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is not built; run python -m paper_2412_14966_amd.build")
        # torch first: it loads its own copy of the HIP runtime under the same
        # soname, and libpvfind must bind to that copy.  Loaded the other way
        # round, the process holds two HIP runtimes and the second one to
        # touch the GPU finds no device.
        import torch  # noqa: F401
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.POINTER
        vp = ctypes.c_void_p
        L.pv_params_default.argtypes = [P(pv_params)]
        L.pv_params_default.restype = None
        L.pv_nbins.argtypes = [P(pv_params)]
        L.pv_nbins.restype = ctypes.c_int32
        common = [P(pv_tracks), vp, ctypes.c_int32, P(pv_beamline), P(pv_params), P(pv_vertices_out),
                  P(pv_track_out)]
        L.pv_find.argtypes = common + [vp]
        L.pv_find_noalloc.argtypes = common + [vp]
        L.pv_find_sched.argtypes = common + [P(pv_schedule), vp]
        L.pv_find_debug.argtypes = common + [P(pv_debug_out), P(pv_schedule), vp]
        for f in (L.pv_find, L.pv_find_sched, L.pv_find_debug):
            f.restype = ctypes.c_int
        L.pv_autotune.argtypes = common + [ctypes.c_int32, ctypes.c_char_p, ctypes.c_char_p, ctypes.c_int32,
                                           P(pv_schedule), P(ctypes.c_double), vp]
        L.pv_autotune.restype = ctypes.c_int
        L.pv_set_schedule.argtypes = [P(pv_schedule)]
        L.pv_get_schedule.argtypes = [P(pv_schedule)]
        L.pv_timing_start.argtypes = []
        L.pv_timing_stop.argtypes = [P(ctypes.c_double), P(ctypes.c_double), P(ctypes.c_int64)]
        L.pv_measure_lds_peak.argtypes = [P(ctypes.c_double), P(ctypes.c_int32), vp]
        L.pv_compact_vertices.argtypes = [vp, vp, ctypes.c_int32, ctypes.c_int32, vp, vp, vp]
        L.pv_last_error.restype = ctypes.c_char_p
        L.pv_version.restype = ctypes.c_char_p
        _lib = L
    return _lib


def pv_last_error() -> str:
    return lib().pv_last_error().decode()


def pv_version() -> str:
    return lib().pv_version().decode()


def _check(rc: int):
    if rc != PV_OK:
        raise PvError(rc, pv_last_error())


def pv_params_default() -> pv_params:
    p = pv_params()
    lib().pv_params_default(ctypes.byref(p))
    return p


def make_params(overrides: Optional[Dict] = None) -> pv_params:
    p = pv_params_default()
    for k, v in (overrides or {}).items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def params_dict(p: pv_params) -> Dict:
    return {name: getattr(p, name) for name, _ in pv_params._fields_}


def pv_nbins(params: Optional[pv_params] = None) -> int:
    return lib().pv_nbins(ctypes.byref(params or pv_params_default()))


def pv_set_schedule(waves_per_team=2, track_capacity=512, persistent=2, teams_per_cu=0):
    _check(lib().pv_set_schedule(ctypes.byref(pv_schedule(waves_per_team, track_capacity, persistent,
                                                          teams_per_cu))))


def pv_get_schedule() -> pv_schedule:
    s = pv_schedule()
    _check(lib().pv_get_schedule(ctypes.byref(s)))
    return s


def pv_timing_start():
    _check(lib().pv_timing_start())


def pv_compact_vertices(out: "Outputs", n_events: int, dense, first, stream=None):
    """Gather the written vertex records of `out` into `dense` (uint8 device
    tensor of at least 64 * n_events * max_vertices bytes); `first` (int32
    device tensor of n_events + 1) receives the per-event offsets and total."""
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_compact_vertices(ctypes.c_void_p(out.vertices.data_ptr()), ctypes.c_void_p(out.n_vertices.data_ptr()),
                                     n_events, out.max_vertices, ctypes.c_void_p(dense.data_ptr()),
                                     ctypes.c_void_p(first.data_ptr()), st))


def pv_measure_lds_peak(stream=None):
    """(LDS read bandwidth in bytes/s, workgroups of the probe launch)."""
    bw, wg = ctypes.c_double(), ctypes.c_int32()
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_measure_lds_peak(ctypes.byref(bw), ctypes.byref(wg), st))
    return bw.value, wg.value


def pv_timing_stop():
    """(main kernel ms, large-event kernel ms, calls) summed over the timed calls."""
    a, b, n = ctypes.c_double(), ctypes.c_double(), ctypes.c_int64()
    _check(lib().pv_timing_stop(ctypes.byref(a), ctypes.byref(b), ctypes.byref(n)))
    return a.value, b.value, n.value


# ---------------------------------------------------------------------------
# device-resident batches (torch tensors)
# ---------------------------------------------------------------------------
@dataclasses.dataclass
class DeviceBatch:
    cols: list                 # 8 float32 device tensors
    offsets: "object"          # int32 device tensor, n_events + 1
    n_events: int
    n_tracks: int
    beamline: tuple


def to_device(batch: synth.TrackBatch, device="cuda") -> DeviceBatch:
    import torch
    # the library takes no null track array, also for a batch without tracks:
    # such a batch gets one unread element per column
    cols = [torch.from_numpy(np.ascontiguousarray(c if c.size else np.zeros(1, dtype=np.float32))).to(device)
            for c in batch.fields()]
    offs = torch.from_numpy(np.ascontiguousarray(batch.offsets, dtype=np.int32)).to(device)
    return DeviceBatch(cols=cols, offsets=offs, n_events=batch.n_events, n_tracks=batch.n_tracks,
                       beamline=tuple(batch.beamline))


@dataclasses.dataclass
class Outputs:
    vertices: "object"         # uint8 device tensor, n_events * max_vertices * 64 bytes
    n_vertices: "object"       # int32 device tensor
    status: "object"           # int32 device tensor
    track_vertex: "object"     # int32 device tensor
    track_weight: "object"     # float32 device tensor
    max_vertices: int


def alloc_outputs(db: DeviceBatch, max_vertices: int, device="cuda") -> Outputs:
    import torch
    ne = max(db.n_events, 1)
    nt = max(db.n_tracks, 1)
    return Outputs(vertices=torch.empty(ne * max_vertices * 64, dtype=torch.uint8, device=device),
                   n_vertices=torch.empty(ne, dtype=torch.int32, device=device),
                   status=torch.empty(ne, dtype=torch.int32, device=device),
                   track_vertex=torch.empty(nt, dtype=torch.int32, device=device),
                   track_weight=torch.empty(nt, dtype=torch.float32, device=device),
                   max_vertices=max_vertices)


def _current_stream():
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


def _args(db: DeviceBatch, out: Outputs, params: pv_params):
    tr = pv_tracks(*[c.data_ptr() for c in db.cols])
    bl = pv_beamline(*[float(v) for v in db.beamline])
    ov = pv_vertices_out(out.vertices.data_ptr(), out.n_vertices.data_ptr(), out.status.data_ptr())
    ot = pv_track_out(out.track_vertex.data_ptr(), out.track_weight.data_ptr())
    return tr, bl, ov, ot


def pv_find(db: DeviceBatch, out: Outputs, params: pv_params, stream=None):
    """Enqueue pv_find on `stream` (default: torch's current stream)."""
    tr, bl, ov, ot = _args(db, out, params)
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_find(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr()), db.n_events, ctypes.byref(bl),
                         ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot), st))


PV_NOALLOC_MAX_EVENTS = 262144


def pv_find_noalloc(db: DeviceBatch, out: Outputs, params: pv_params, stream=None):
    """Enqueue pv_find_noalloc (no device allocation; at most
    PV_NOALLOC_MAX_EVENTS events; calls overlapping on one device race)."""
    tr, bl, ov, ot = _args(db, out, params)
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_find_noalloc(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr()), db.n_events,
                                 ctypes.byref(bl), ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot), st))


def pv_find_sched(db: DeviceBatch, out: Outputs, params: pv_params, schedule: pv_schedule, stream=None):
    tr, bl, ov, ot = _args(db, out, params)
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_find_sched(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr()), db.n_events,
                               ctypes.byref(bl), ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot),
                               ctypes.byref(schedule), st))


def pv_autotune(db: DeviceBatch, out: Outputs, params: pv_params, reps: int = 5, cache_path: Optional[str] = None,
                key: Optional[str] = None, force: bool = False, stream=None):
    """Time every schedule on this batch and make the fastest the default.
    Returns (schedule dict, microseconds per launch; 0 when read from the cache)."""
    tr, bl, ov, ot = _args(db, out, params)
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    best = pv_schedule()
    us = ctypes.c_double()
    _check(lib().pv_autotune(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr()), db.n_events,
                             ctypes.byref(bl), ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot), int(reps),
                             cache_path.encode() if cache_path else None, key.encode() if key else None,
                             1 if force else 0, ctypes.byref(best), ctypes.byref(us), st))
    return (dict(waves_per_team=best.waves_per_team, track_capacity=best.track_capacity,
                 persistent=best.persistent, teams_per_cu=best.teams_per_cu), us.value)


@dataclasses.dataclass
class DebugOutputs:
    hist: "object"
    clusters: "object"
    n_clusters: "object"
    zpoca: "object"
    sigma: "object"
    bin: "object"
    stage_cycles: "object"


def pv_find_debug(db: DeviceBatch, out: Outputs, params: pv_params, schedule: Optional[pv_schedule] = None,
                  stream=None) -> DebugOutputs:
    import torch
    dev = out.n_vertices.device
    nb = pv_nbins(params)
    ne, nt = max(db.n_events, 1), max(db.n_tracks, 1)
    d = DebugOutputs(hist=torch.empty(ne * nb, dtype=torch.int32, device=dev),
                     clusters=torch.empty(ne * out.max_vertices * 32, dtype=torch.uint8, device=dev),
                     n_clusters=torch.empty(ne, dtype=torch.int32, device=dev),
                     zpoca=torch.empty(nt, dtype=torch.float32, device=dev),
                     sigma=torch.empty(nt, dtype=torch.float32, device=dev),
                     bin=torch.empty(nt, dtype=torch.int32, device=dev),
                     stage_cycles=torch.zeros(ne * 8, dtype=torch.int32, device=dev))
    dbg = pv_debug_out(d.hist.data_ptr(), d.clusters.data_ptr(), d.n_clusters.data_ptr(), d.zpoca.data_ptr(),
                       d.sigma.data_ptr(), d.bin.data_ptr(), d.stage_cycles.data_ptr())
    tr, bl, ov, ot = _args(db, out, params)
    st = ctypes.c_void_p(stream) if stream is not None else _current_stream()
    _check(lib().pv_find_debug(ctypes.byref(tr), ctypes.c_void_p(db.offsets.data_ptr()), db.n_events,
                               ctypes.byref(bl), ctypes.byref(params), ctypes.byref(ov), ctypes.byref(ot),
                               ctypes.byref(dbg), ctypes.byref(schedule) if schedule is not None else None, st))
    return d


@dataclasses.dataclass
class HostResult:
    n_vertices: np.ndarray
    status: np.ndarray
    vertices: np.ndarray       # (n_events, max_vertices) VERTEX_DTYPE
    track_vertex: np.ndarray
    track_weight: np.ndarray
    hist: Optional[np.ndarray] = None
    clusters: Optional[np.ndarray] = None
    n_clusters: Optional[np.ndarray] = None
    zpoca: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    bin: Optional[np.ndarray] = None
    stage_cycles: Optional[np.ndarray] = None


def to_host(db: DeviceBatch, out: Outputs, dbg: Optional[DebugOutputs] = None, nb: int = 0) -> HostResult:
    ne, nt, mv = db.n_events, db.n_tracks, out.max_vertices
    vt = out.vertices.cpu().numpy()[:ne * mv * 64].view(VERTEX_DTYPE).reshape(ne, mv)
    r = HostResult(n_vertices=out.n_vertices.cpu().numpy()[:ne], status=out.status.cpu().numpy()[:ne], vertices=vt,
                   track_vertex=out.track_vertex.cpu().numpy()[:nt], track_weight=out.track_weight.cpu().numpy()[:nt])
    if dbg is not None:
        r.hist = dbg.hist.cpu().numpy()[:ne * nb].reshape(ne, nb)
        r.clusters = dbg.clusters.cpu().numpy()[:ne * mv * 32].view(CLUSTER_DTYPE).reshape(ne, mv)
        r.n_clusters = dbg.n_clusters.cpu().numpy()[:ne]
        r.zpoca = dbg.zpoca.cpu().numpy()[:nt]
        r.sigma = dbg.sigma.cpu().numpy()[:nt]
        r.bin = dbg.bin.cpu().numpy()[:nt]
        r.stage_cycles = dbg.stage_cycles.cpu().numpy()[:ne * 8].view(np.uint32).reshape(ne, 8)
    return r


def run(batch: synth.TrackBatch, params: Optional[Dict] = None, schedule: Optional[Dict] = None, debug=False,
        device="cuda") -> HostResult:
    """Convenience: copy a batch to the device, run, synchronise, copy back."""
    import torch
    p = make_params(params)
    db = to_device(batch, device)
    out = alloc_outputs(db, p.max_vertices_per_event, device)
    sch = pv_schedule(**schedule) if schedule else None
    if debug:
        d = pv_find_debug(db, out, p, sch)
    elif sch is not None:
        pv_find_sched(db, out, p, sch)
        d = None
    else:
        pv_find(db, out, p)
        d = None
    torch.cuda.synchronize()
    return to_host(db, out, d, pv_nbins(p))


# ---------------------------------------------------------------------------
# serving (continuous batching), see pv_server_* in include/pvfind.h
# ---------------------------------------------------------------------------
class pv_server_config(ctypes.Structure):
    _fields_ = [("max_events_per_batch", ctypes.c_int32), ("max_tracks_per_batch", ctypes.c_int32),
                ("n_slots", ctypes.c_int32), ("n_streams", ctypes.c_int32),
                ("device_budget_bytes", ctypes.c_int64), ("max_wait_us", ctypes.c_int32),
                ("use_graphs", ctypes.c_int32)]


class pv_request(ctypes.Structure):
    _fields_ = [(n, ctypes.c_void_p) for n in ("x", "y", "z", "tx", "ty", "cov_xx", "cov_xtx", "cov_txtx")] + \
               [("n_tracks", ctypes.c_int32), ("vertices", ctypes.c_void_p), ("track_vertex", ctypes.c_void_p),
                ("track_weight", ctypes.c_void_p)]


class pv_completion(ctypes.Structure):
    _fields_ = [("tag", ctypes.c_uint64), ("status", ctypes.c_int32), ("n_vertices", ctypes.c_int32),
                ("t_arrival_ns", ctypes.c_int64), ("t_done_ns", ctypes.c_int64)]


class pv_server_stats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64), ("rejected_busy", ctypes.c_int64),
                ("batches", ctypes.c_int64), ("mean_batch_events", ctypes.c_double),
                ("device_bytes", ctypes.c_int64)]


COMPLETION_DTYPE = np.dtype([("tag", "<u8"), ("status", "<i4"), ("n_vertices", "<i4"), ("t_arrival_ns", "<i8"),
                             ("t_done_ns", "<i8")])
assert COMPLETION_DTYPE.itemsize == ctypes.sizeof(pv_completion)

_server_ready = False


def _server_lib():
    global _server_ready
    L = lib()
    if not _server_ready:
        P = ctypes.POINTER
        L.pv_clock_ns.restype = ctypes.c_int64
        L.pv_server_config_default.argtypes = [P(pv_server_config)]
        L.pv_server_config_default.restype = None
        L.pv_server_create.argtypes = [P(ctypes.c_void_p), P(pv_params), P(pv_beamline), P(pv_server_config),
                                       P(pv_schedule)]
        L.pv_server_submit.argtypes = [ctypes.c_void_p, P(pv_request), ctypes.c_uint64, ctypes.c_int64]
        L.pv_server_poll.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32, ctypes.c_int32]
        L.pv_server_drain.argtypes = [ctypes.c_void_p, ctypes.c_int32]
        L.pv_server_replay.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int32,
                                       ctypes.c_void_p]
        L.pv_server_get_stats.argtypes = [ctypes.c_void_p, P(pv_server_stats)]
        L.pv_server_destroy.argtypes = [ctypes.c_void_p]
        _server_ready = True
    return L


def pv_server_config_default(**overrides) -> pv_server_config:
    c = pv_server_config()
    _server_lib().pv_server_config_default(ctypes.byref(c))
    for k, v in overrides.items():
        if not hasattr(c, k):
            raise KeyError(k)
        setattr(c, k, v)
    return c


class HostEvents:
    """Host-side requests for every event of a TrackBatch, with output arrays."""

    def __init__(self, batch: synth.TrackBatch, max_vertices: int):
        self.batch = batch
        self.cols = [np.ascontiguousarray(c, dtype=np.float32) for c in batch.fields()]
        ne, nt = batch.n_events, batch.n_tracks
        self.vertices = np.zeros((max(ne, 1), max_vertices), dtype=VERTEX_DTYPE)
        self.track_vertex = np.full(max(nt, 1), -7, dtype=np.int32)
        self.track_weight = np.full(max(nt, 1), -7.0, dtype=np.float32)
        self.requests = (pv_request * max(ne, 1))()
        for e in range(ne):
            a, n = int(batch.offsets[e]), int(batch.offsets[e + 1] - batch.offsets[e])
            r = self.requests[e]
            for k, name in enumerate(("x", "y", "z", "tx", "ty", "cov_xx", "cov_xtx", "cov_txtx")):
                setattr(r, name, self.cols[k].ctypes.data + 4 * a)
            r.n_tracks = n
            r.vertices = self.vertices.ctypes.data + e * max_vertices * 64
            r.track_vertex = self.track_vertex.ctypes.data + 4 * a
            r.track_weight = self.track_weight.ctypes.data + 4 * a


class Server:
    """pv_server_*: continuous batching of events submitted from the host."""

    def __init__(self, params: pv_params, beamline=(0.0, 0.0, 0.0, 0.0), config: Optional[pv_server_config] = None,
                 schedule: Optional[pv_schedule] = None):
        L = _server_lib()
        self.params = params
        self.config = config or pv_server_config_default()
        h = ctypes.c_void_p()
        bl = pv_beamline(*[float(v) for v in beamline])
        _check(L.pv_server_create(ctypes.byref(h), ctypes.byref(params), ctypes.byref(bl),
                                  ctypes.byref(self.config), ctypes.byref(schedule) if schedule else None))
        self.handle = h

    def submit(self, req: pv_request, tag: int, t_arrival_ns: int = 0) -> int:
        """Returns PV_OK or PV_EBUSY; raises on other errors."""
        rc = _server_lib().pv_server_submit(self.handle, ctypes.byref(req), tag, t_arrival_ns)
        if rc not in (PV_OK, PV_EBUSY):
            _check(rc)
        return rc

    def poll(self, max_out: int = 1024, timeout_us: int = 0) -> np.ndarray:
        out = np.zeros(max_out, dtype=COMPLETION_DTYPE)
        k = _server_lib().pv_server_poll(self.handle, out.ctypes.data, max_out, timeout_us)
        if k < 0:
            _check(k)
        return out[:k]

    def drain(self, timeout_ms: int = -1):
        _check(_server_lib().pv_server_drain(self.handle, timeout_ms))

    def replay(self, events: HostEvents, t_offset_ns: np.ndarray) -> np.ndarray:
        n = events.batch.n_events
        offs = np.ascontiguousarray(t_offset_ns, dtype=np.int64)
        if offs.shape != (n,):
            raise ValueError(f"replay needs one arrival offset per event ({n}), got {offs.shape}")
        if n and (offs.min() < 0 or np.any(np.diff(offs) < 0)):
            raise ValueError("arrival offsets must be non-negative and non-decreasing")
        out = np.zeros(max(n, 1), dtype=COMPLETION_DTYPE)
        _check(_server_lib().pv_server_replay(self.handle, ctypes.addressof(events.requests), offs.ctypes.data, n,
                                              out.ctypes.data))
        return out[:n]

    def stats(self) -> dict:
        st = pv_server_stats()
        _check(_server_lib().pv_server_get_stats(self.handle, ctypes.byref(st)))
        return {name: getattr(st, name) for name, _ in pv_server_stats._fields_}

    def close(self):
        if self.handle:
            _check(_server_lib().pv_server_destroy(self.handle))
            self.handle = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()


def pv_clock_ns() -> int:
    return _server_lib().pv_clock_ns()
