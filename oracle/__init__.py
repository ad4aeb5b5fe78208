"""Python access to the CPU oracle (``liboracle.so`` built from pv_oracle.c).

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the
CPU-baseline leg of the benchmark use this module; the product path never
imports it.  It shares no code with the HIP library.
"""
from __future__ import annotations

import ctypes
import dataclasses
import os
import subprocess
from typing import Dict, Optional

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "pv_oracle.c")
# PV_ORACLE_LIB names another build of the oracle (the mutation test loads
# planted-mistake builds this way); it is loaded as it is, never rebuilt
_LIB_OVERRIDE = os.environ.get("PV_ORACLE_LIB")
_LIB = _LIB_OVERRIDE or os.path.join(_HERE, "liboracle.so")

TR_HIST, TR_ASSOC, TR_NONFINITE = 1, 2, 4
EV_NONFINITE_INPUT, EV_TOO_MANY_TRACKS, EV_VERTEX_OVERFLOW, EV_OFFSETS_INVALID = 1, 2, 4, 8
EV_FIT_FAILED = 16
VX_NOT_CONVERGED = 1


GCC_FLAGS = ["-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fexcess-precision=standard",
             "-fopenmp", "-fPIC", "-shared", "-Wall", "-Wextra"]


def build(force: bool = True, src: str = _SRC, out: Optional[str] = None) -> str:
    """Compile liboracle.so with gcc (binary32 stage needs -ffp-contract=off)."""
    out = out or os.path.join(_HERE, "liboracle.so")
    if force or not os.path.exists(out):
        tmp = out + ".tmp"
        subprocess.check_call(["gcc", *GCC_FLAGS, "-I", _HERE, "-o", tmp, src, "-lm"])
        os.replace(tmp, out)
    return out


class OrcParams(ctypes.Structure):
    _fields_ = [
        ("z_min", ctypes.c_float), ("z_max", ctypes.c_float), ("dz", ctypes.c_float), ("z_gas", ctypes.c_float),
        ("sigma_max_pp", ctypes.c_float), ("sigma_max_gas", ctypes.c_float), ("u0", ctypes.c_float),
        ("frac_bits", ctypes.c_int),
        ("proto_thr", ctypes.c_int), ("dip_prom", ctypes.c_int), ("min_int_pp", ctypes.c_int),
        ("min_int_gas", ctypes.c_int),
        ("part_min_pp", ctypes.c_int), ("part_min_gas", ctypes.c_int), ("pv_min_pp", ctypes.c_int),
        ("pv_min_gas", ctypes.c_int),
        ("max_iter", ctypes.c_int),
        ("chi2_max", ctypes.c_double), ("conv_dchi2", ctypes.c_double), ("conv_dz", ctypes.c_double),
        ("max_rho_pp", ctypes.c_double), ("sing_ratio", ctypes.c_double),
        ("max_tracks", ctypes.c_int), ("max_vertices", ctypes.c_int),
        ("assoc_mode", ctypes.c_int), ("chi2_max_mv", ctypes.c_double), ("chi2_window_mv", ctypes.c_double),
        ("conv_dz_mv", ctypes.c_double), ("dup_ratio", ctypes.c_double), ("w_count_mv", ctypes.c_double),
        ("peak_mode", ctypes.c_int), ("tie_rel", ctypes.c_double), ("iter_override_bin", ctypes.c_int),
        ("iter_override_n", ctypes.c_int),
    ]


class OrcCluster(ctypes.Structure):
    _fields_ = [("lo", ctypes.c_int), ("hi", ctypes.c_int), ("peak", ctypes.c_int), ("z_seed", ctypes.c_double),
                ("kept", ctypes.c_int), ("n_assoc", ctypes.c_int), ("own_lo", ctypes.c_int),
                ("own_hi", ctypes.c_int), ("n_near_cut", ctypes.c_int)]


class OrcVertex(ctypes.Structure):
    _fields_ = [("x", ctypes.c_double), ("y", ctypes.c_double), ("z", ctypes.c_double),
                ("cov", ctypes.c_double * 6), ("chi2", ctypes.c_double), ("ndof", ctypes.c_double),
                ("z_seed", ctypes.c_double), ("conv_margin", ctypes.c_double), ("dchi2", ctypes.c_double),
                ("n_tracks", ctypes.c_int), ("bin_lo", ctypes.c_int), ("bin_hi", ctypes.c_int),
                ("peak_bin", ctypes.c_int), ("n_iter", ctypes.c_int), ("flags", ctypes.c_int),
                ("n_near", ctypes.c_int), ("dup_margin", ctypes.c_double)]


_VERTEX_DTYPE = np.dtype([("x", "f8"), ("y", "f8"), ("z", "f8"), ("cov", "f8", (6,)), ("chi2", "f8"),
                          ("ndof", "f8"), ("z_seed", "f8"), ("conv_margin", "f8"), ("dchi2", "f8"),
                          ("n_tracks", "i4"),
                          ("bin_lo", "i4"), ("bin_hi", "i4"), ("peak_bin", "i4"), ("n_iter", "i4"),
                          ("flags", "i4"), ("n_near", "i4"), ("dup_margin", "f8")], align=True)
_CLUSTER_DTYPE = np.dtype([("lo", "i4"), ("hi", "i4"), ("peak", "i4"), ("z_seed", "f8"), ("kept", "i4"),
                           ("n_assoc", "i4"), ("own_lo", "i4"), ("own_hi", "i4"), ("n_near_cut", "i4")],
                          align=True)
assert _VERTEX_DTYPE.itemsize == ctypes.sizeof(OrcVertex)
assert _CLUSTER_DTYPE.itemsize == ctypes.sizeof(OrcCluster)

_lib = None


def lib():
    global _lib
    if _lib is None:
        if not _LIB_OVERRIDE and (not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC)):
            build()
        L = ctypes.CDLL(_LIB)
        P = ctypes.POINTER
        fp, ip, dp = P(ctypes.c_float), P(ctypes.c_int), P(ctypes.c_double)
        L.orc_params_default.argtypes = [P(OrcParams)]
        L.orc_nbins.argtypes = [P(OrcParams)]
        L.orc_gas_bin.argtypes = [P(OrcParams)]
        L.orc_project.argtypes = [fp, fp, P(OrcParams), fp, fp, ip]
        L.orc_edge_code.argtypes = [ctypes.c_float, ctypes.c_float, ctypes.c_float, ctypes.c_int]
        L.orc_hist_event.argtypes = [ctypes.c_void_p * 8, ctypes.c_int, fp, P(OrcParams), ip, ip]
        L.orc_peak_search.argtypes = [ip, P(OrcParams), ctypes.c_void_p, ctypes.c_int, ip]
        L.orc_seed_z.argtypes = [ip, ctypes.c_int, ctypes.c_int, P(OrcParams)]
        L.orc_seed_z.restype = ctypes.c_double
        L.orc_partition.argtypes = [ctypes.c_void_p, ctypes.c_int, ip, P(OrcParams)]
        L.orc_fit.argtypes = [ctypes.c_void_p * 8, ip, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                              ctypes.c_double, P(OrcParams), P(OrcVertex), dp]
        L.orc_mv_weight.argtypes = [ctypes.c_double, ctypes.c_double, ctypes.c_double]
        L.orc_mv_weight.restype = ctypes.c_double
        L.orc_fit_mv.argtypes = [ctypes.c_void_p * 8, ip, dp, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                 ctypes.c_double, P(OrcParams), P(OrcVertex), dp]
        L.orc_find.argtypes = [ctypes.c_void_p * 8, ip, ctypes.c_int, fp, P(OrcParams), ip, ip, ctypes.c_void_p,
                               ip, dp, ip, ctypes.c_void_p, ip, fp, fp, ip, ctypes.c_int]
        L.orc_max_threads.argtypes = []
        _lib = L
    return _lib


def _ptr(a: Optional[np.ndarray], ctype):
    if a is None:
        return None
    return a.ctypes.data_as(ctypes.POINTER(ctype))


def default_params() -> Dict[str, float]:
    p = OrcParams()
    lib().orc_params_default(ctypes.byref(p))
    return {name: getattr(p, name) for name, _ in OrcParams._fields_}


def make_params(overrides: Optional[Dict[str, float]] = None) -> OrcParams:
    p = OrcParams()
    lib().orc_params_default(ctypes.byref(p))
    for k, v in (overrides or {}).items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


# parameter names of the HIP library that differ from the oracle's
_LIBRARY_NAMES = {"max_tracks_per_event": "max_tracks", "max_vertices_per_event": "max_vertices"}


def params_from_fields(fields: Dict) -> Dict:
    """Oracle parameters holding the values of a parameter mapping that uses
    the HIP library's field names (fields the oracle has no use for, such as
    the binary64-inversion threshold of the GPU, are ignored)."""
    names = {n for n, _ in OrcParams._fields_}
    out = {}
    for k, v in fields.items():
        k2 = _LIBRARY_NAMES.get(k, k)
        if k2 in names:
            out[k2] = v
    return out


def nbins(params: Optional[Dict] = None) -> int:
    return lib().orc_nbins(ctypes.byref(make_params(params)))


def gas_bin(params: Optional[Dict] = None) -> int:
    return lib().orc_gas_bin(ctypes.byref(make_params(params)))


def _beam(beamline) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(beamline, dtype=np.float32).reshape(4))


def project(track, beamline=(0, 0, 0, 0), params=None):
    """Eq. 1 and Eq. 3 for one track.  Returns (flags, zpoca, sigma, bin)."""
    t = np.ascontiguousarray(np.asarray(track, dtype=np.float32).reshape(8))
    b = _beam(beamline)
    zp, sg, bn = ctypes.c_float(), ctypes.c_float(), ctypes.c_int()
    fl = lib().orc_project(_ptr(t, ctypes.c_float), _ptr(b, ctypes.c_float), ctypes.byref(make_params(params)),
                           ctypes.byref(zp), ctypes.byref(sg), ctypes.byref(bn))
    return fl, zp.value, sg.value, bn.value


def edge_code(e: float, zp: float, sw: float, frac_bits: int = 16) -> int:
    return lib().orc_edge_code(ctypes.c_float(e), ctypes.c_float(zp), ctypes.c_float(sw), frac_bits)


def _track_ptrs(cols):
    arr = (ctypes.c_void_p * 8)()
    keep = []
    for k, c in enumerate(cols):
        c = np.ascontiguousarray(c, dtype=np.float32)
        keep.append(c)
        arr[k] = c.ctypes.data
    return arr, keep


def hist_event(tracks: np.ndarray, beamline=(0, 0, 0, 0), params=None):
    """Histogram h and per-bin associable-track counts c of one event given as
    an (n, 8) array of track states."""
    P = make_params(params)
    nb = lib().orc_nbins(ctypes.byref(P))
    t = np.asarray(tracks, dtype=np.float32).reshape(-1, 8)
    arr, keep = _track_ptrs([t[:, k] for k in range(8)])
    h = np.zeros(nb, dtype=np.int32)
    c = np.zeros(nb, dtype=np.int32)
    lib().orc_hist_event(arr, t.shape[0], _ptr(_beam(beamline), ctypes.c_float), ctypes.byref(P),
                         _ptr(h, ctypes.c_int), _ptr(c, ctypes.c_int))
    del keep
    return h, c


def peak_search(h: np.ndarray, params=None, max_out: int = 4096):
    """Seed clusters of a histogram: structured array (lo, hi, peak, z_seed, ...)
    and the overflow flag."""
    P = make_params(params)
    h = np.ascontiguousarray(h, dtype=np.int32)
    assert h.shape[0] == lib().orc_nbins(ctypes.byref(P))
    out = np.zeros(max_out, dtype=_CLUSTER_DTYPE)
    ov = ctypes.c_int()
    n = lib().orc_peak_search(_ptr(h, ctypes.c_int), ctypes.byref(P), out.ctypes.data, max_out, ctypes.byref(ov))
    return out[:n].copy(), bool(ov.value)


def seed_z(h: np.ndarray, i: int, params=None) -> float:
    P = make_params(params)
    h = np.ascontiguousarray(h, dtype=np.int32)
    return lib().orc_seed_z(_ptr(h, ctypes.c_int), h.shape[0], int(i), ctypes.byref(P))


def partition(clusters: np.ndarray, c: np.ndarray, params=None) -> np.ndarray:
    """Association step on a cluster list (structured array from peak_search)
    and per-bin track counts; returns the updated cluster array."""
    P = make_params(params)
    cl = np.ascontiguousarray(clusters.copy(), dtype=_CLUSTER_DTYPE)
    c = np.ascontiguousarray(c, dtype=np.int32)
    lib().orc_partition(cl.ctypes.data if cl.shape[0] else None, cl.shape[0], _ptr(c, ctypes.c_int),
                        ctypes.byref(P))
    return cl


def fit(tracks: np.ndarray, seed, params=None):
    """Adaptive fit of all tracks of an (n, 8) array from seed (x, y, z).
    Returns (failed, vertex record, weights)."""
    P = make_params(params)
    t = np.asarray(tracks, dtype=np.float32).reshape(-1, 8)
    n = t.shape[0]
    arr, keep = _track_ptrs([t[:, k] for k in range(8)])
    idx = np.arange(n, dtype=np.int32)
    w = np.zeros(max(n, 1), dtype=np.float64)
    v = OrcVertex()
    bad = lib().orc_fit(arr, _ptr(idx, ctypes.c_int), n, float(seed[0]), float(seed[1]), float(seed[2]),
                        ctypes.byref(P), ctypes.byref(v), _ptr(w, ctypes.c_double))
    rec = np.frombuffer(bytes(v), dtype=_VERTEX_DTYPE)[0]
    del keep
    return bool(bad), rec, w[:n].copy()


def mv_weight(chi2: float, others: float = 0.0, chi2_max: float = 4.0) -> float:
    """Eq. 18 for one track: chi2 relative to this candidate, the sum of
    exp(-chi2_k / 2) over the other candidates."""
    return lib().orc_mv_weight(float(chi2), float(others), float(chi2_max))


def fit_mv(tracks: np.ndarray, others, seed, params=None):
    """Fit with the weights of Eq. 18 (GPU variant) of all tracks of an (n, 8)
    array from seed (x, y, z); others[k] is track k's sum of exp(-chi2 / 2)
    over the other candidates.  Returns (failed, vertex record, weights)."""
    P = make_params(params)
    t = np.asarray(tracks, dtype=np.float32).reshape(-1, 8)
    n = t.shape[0]
    arr, keep = _track_ptrs([t[:, k] for k in range(8)])
    idx = np.arange(n, dtype=np.int32)
    oth = np.ascontiguousarray(np.broadcast_to(np.asarray(others, dtype=np.float64), (n,)))
    w = np.zeros(max(n, 1), dtype=np.float64)
    v = OrcVertex()
    bad = lib().orc_fit_mv(arr, _ptr(idx, ctypes.c_int), _ptr(oth, ctypes.c_double), n, float(seed[0]),
                           float(seed[1]), float(seed[2]), ctypes.byref(P), ctypes.byref(v),
                           _ptr(w, ctypes.c_double))
    rec = np.frombuffer(bytes(v), dtype=_VERTEX_DTYPE)[0]
    del keep
    return bool(bad), rec, w[:n].copy()


@dataclasses.dataclass
class OracleResult:
    n_vertices: np.ndarray      # (n_events,) int32
    status: np.ndarray          # (n_events,) int32
    vertices: np.ndarray        # (n_events, max_vertices) structured
    track_vertex: np.ndarray    # (n_tracks,) int32
    track_weight: np.ndarray    # (n_tracks,) float64
    hist: Optional[np.ndarray] = None
    clusters: Optional[np.ndarray] = None
    n_clusters: Optional[np.ndarray] = None
    zpoca: Optional[np.ndarray] = None
    sigma: Optional[np.ndarray] = None
    bin: Optional[np.ndarray] = None
    params: Optional[Dict] = None   # the parameter overrides this result was computed with


def find(batch, params=None, debug: bool = False, n_threads: int = 0) -> OracleResult:
    """Run the whole path on a TrackBatch (paper_2412_14966_amd.synth)."""
    P = make_params(params)
    L = lib()
    nb = L.orc_nbins(ctypes.byref(P))
    ne = batch.n_events
    nt = int(batch.offsets[-1]) if ne >= 0 else 0
    arr, keep = _track_ptrs(batch.fields())
    offs = np.ascontiguousarray(batch.offsets, dtype=np.int32)
    maxv = P.max_vertices
    nv = np.zeros(max(ne, 1), np.int32)
    st = np.zeros(max(ne, 1), np.int32)
    vtx = np.zeros(max(ne, 1) * maxv, dtype=_VERTEX_DTYPE)
    tv = np.full(max(nt, 1), -1, np.int32)
    tw = np.zeros(max(nt, 1), np.float64)
    hist = np.zeros(max(ne, 1) * nb, np.int32) if debug else None
    cls = np.zeros(max(ne, 1) * maxv, dtype=_CLUSTER_DTYPE) if debug else None
    ncl = np.zeros(max(ne, 1), np.int32) if debug else None
    zp = np.zeros(max(nt, 1), np.float32) if debug else None
    sg = np.zeros(max(nt, 1), np.float32) if debug else None
    bn = np.full(max(nt, 1), -1, np.int32) if debug else None
    rc = L.orc_find(arr, _ptr(offs, ctypes.c_int), ne, _ptr(_beam(batch.beamline), ctypes.c_float),
                    ctypes.byref(P), _ptr(nv, ctypes.c_int), _ptr(st, ctypes.c_int), vtx.ctypes.data,
                    _ptr(tv, ctypes.c_int), _ptr(tw, ctypes.c_double), _ptr(hist, ctypes.c_int),
                    cls.ctypes.data if cls is not None else None, _ptr(ncl, ctypes.c_int),
                    _ptr(zp, ctypes.c_float), _ptr(sg, ctypes.c_float), _ptr(bn, ctypes.c_int), int(n_threads))
    del keep
    if rc != 0:
        raise ValueError("oracle rejected the arguments")
    res = OracleResult(n_vertices=nv[:ne], status=st[:ne], vertices=vtx[:ne * maxv].reshape(ne, maxv),
                       track_vertex=tv[:nt], track_weight=tw[:nt], params=dict(params or {}))
    if debug:
        res.hist = hist[:ne * nb].reshape(ne, nb)
        res.clusters = cls[:ne * maxv].reshape(ne, maxv)
        res.n_clusters = ncl[:ne]
        res.zpoca, res.sigma, res.bin = zp[:nt], sg[:nt], bn[:nt]
    return res


def max_threads() -> int:
    return lib().orc_max_threads()
