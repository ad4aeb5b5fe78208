"""Seeded synthetic VELO-track events for primary-vertex finding.

This module only draws inputs: it places true interaction points and emits
straight-line track states around them.  It contains none of the
vertex-finding arithmetic (no point-of-closest-approach, no histogram, no
fit), so both the HIP path and the CPU oracle can consume what it writes.

The shapes follow the paper's description of the interaction regions and its
track model; the LHCb simulated samples themselves are not available, so these
distributions stand in for them:

* pp interactions: the visible-interaction count per crossing is Poisson(mu),
  mu = 5 for Run 3 (Sec. 1).  The interaction region is long in z and narrow
  in x and y (Sec. 3, interaction-region discussion); here z ~ N(0, 45 mm) and
  x, y ~ N(0, 0.03 mm).
* p-gas interactions (SMOG2, Sec. 4.2): z uniform over the installed cell,
  [-541, -341] mm (the design cell [-500, -300] mm shifted by the ~4 cm the
  paper's footnote mentions), with fewer tracks per vertex.
* Tracks are straight lines (no magnetic field in the VELO, Sec. 2) with state
  (x, y, tx, ty) at z_trk and a covariance in which x and y are uncorrelated
  and of identical magnitude (Sec. 3.1).  Here the state is given at the z of
  the track origin, smeared transversely by sigma_xy ~ U(0.01, 0.05) mm, so the
  z uncertainty along the beam is sigma_xy / |t| as Eq. (3) states.
* 10 % of tracks start displaced from their vertex by an Exp(1 mm) flight
  distance along their direction (secondary decays).

Every event is drawn from its own PCG64 stream keyed by
SeedSequence([2412, 14966, config_id, event_id]) so that any single event can
be regenerated alone (needed by the served-mode "alone vs in the mix" check).
"""
from __future__ import annotations

import dataclasses
import math
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

TRACK_FIELDS = ("x", "y", "z", "tx", "ty", "cov_xx", "cov_xtx", "cov_txtx")

# Named workloads.  ``mu`` is the mean number of visible pp interactions per
# event; ``mu_loguniform`` draws mu per event as exp(U(0, ln 40)); ``gas_mu``
# is the mean number of beam-gas vertices per event.
WORKLOADS: Dict[str, dict] = {
    "pp_mu5_100ev": dict(config_id=1, n_events=100, mu=5.0, gas_mu=0.0),
    "pp_mu5_10kev": dict(config_id=2, n_events=10_000, mu=5.0, gas_mu=0.0),
    "pp_mu5_gas_50kev": dict(config_id=3, n_events=50_000, mu=5.0, gas_mu=0.5),
    "pp_mu40_20kev": dict(config_id=4, n_events=20_000, mu=40.0, gas_mu=0.0),
    "served_mulog_200kev": dict(config_id=5, n_events=200_000, mu=None, gas_mu=0.0,
                                mu_loguniform=(1.0, 40.0)),
}

PP_Z_SIGMA = 45.0          # mm
PP_XY_SIGMA = 0.03         # mm
PP_TRK_NB = (3, 3.0 / 28.0)    # negative_binomial(n, p): mean 25, k = 3
GAS_TRK_NB = (2, 2.0 / 10.0)   # mean 8, k = 2
GAS_Z_RANGE = (-541.0, -341.0)  # mm
SLOPE_SIGMA = 0.3
SIGMA_XY_RANGE = (0.01, 0.05)  # mm
DISPLACED_FRACTION = 0.10
DISPLACED_MEAN_LENGTH = 1.0    # mm


@dataclasses.dataclass
class TrackBatch:
    """Structure-of-arrays track states for a batch of events.

    Track k of event e is index ``offsets[e] + k``.  All track arrays are
    float32; ``offsets`` is int32 with ``n_events + 1`` entries.
    """

    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    tx: np.ndarray
    ty: np.ndarray
    cov_xx: np.ndarray
    cov_xtx: np.ndarray
    cov_txtx: np.ndarray
    offsets: np.ndarray
    beamline: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0)
    # truth, per event: list of (n_pv, 4) arrays (x, y, z, is_gas) and per-track pv index
    truth_pvs: Optional[List[np.ndarray]] = None
    truth_pv_of_track: Optional[np.ndarray] = None
    truth_ntracks: Optional[List[np.ndarray]] = None

    @property
    def n_events(self) -> int:
        return int(self.offsets.shape[0] - 1)

    @property
    def n_tracks(self) -> int:
        return int(self.offsets[-1])

    def fields(self) -> List[np.ndarray]:
        return [getattr(self, f) for f in TRACK_FIELDS]

    def event(self, e: int) -> "TrackBatch":
        """A one-event batch holding event ``e``."""
        return self.select([e])

    def select(self, events: Sequence[int]) -> "TrackBatch":
        """A batch holding the listed events, in the listed order."""
        events = [int(e) for e in events]
        pieces = {f: [] for f in TRACK_FIELDS}
        counts = []
        for e in events:
            a, b = int(self.offsets[e]), int(self.offsets[e + 1])
            for f in TRACK_FIELDS:
                pieces[f].append(getattr(self, f)[a:b])
            counts.append(b - a)
        offs = np.zeros(len(events) + 1, dtype=np.int32)
        offs[1:] = np.cumsum(counts, dtype=np.int64).astype(np.int32)
        arrays = {f: (np.concatenate(pieces[f]) if pieces[f] else np.zeros(0, np.float32)).astype(np.float32)
                  for f in TRACK_FIELDS}
        tp = [self.truth_pvs[e] for e in events] if self.truth_pvs is not None else None
        tn = [self.truth_ntracks[e] for e in events] if self.truth_ntracks is not None else None
        tpt = None
        if self.truth_pv_of_track is not None:
            tpt = np.concatenate([self.truth_pv_of_track[int(self.offsets[e]):int(self.offsets[e + 1])]
                                  for e in events]) if events else np.zeros(0, np.int32)
        return TrackBatch(offsets=offs, beamline=self.beamline, truth_pvs=tp,
                          truth_pv_of_track=tpt, truth_ntracks=tn, **arrays)


def event_rng(config_id: int, event_id: int) -> np.random.Generator:
    ss = np.random.SeedSequence([2412, 14966, int(config_id), int(event_id)])
    return np.random.Generator(np.random.PCG64(ss))


def _draw_event(rng: np.random.Generator, mu: float, gas_mu: float,
                beamline: Tuple[float, float, float, float], slope_cov: bool):
    xb, yb, txb, tyb = beamline
    n_pp = int(rng.poisson(mu))
    pz = rng.normal(0.0, PP_Z_SIGMA, n_pp)
    px = rng.normal(0.0, PP_XY_SIGMA, n_pp)
    py = rng.normal(0.0, PP_XY_SIGMA, n_pp)
    nt = 1 + rng.negative_binomial(PP_TRK_NB[0], PP_TRK_NB[1], n_pp)
    gas = np.zeros(n_pp, dtype=bool)
    if gas_mu > 0.0:
        n_gas = int(rng.poisson(gas_mu))
        gz = rng.uniform(GAS_Z_RANGE[0], GAS_Z_RANGE[1], n_gas)
        gx = rng.normal(0.0, PP_XY_SIGMA, n_gas)
        gy = rng.normal(0.0, PP_XY_SIGMA, n_gas)
        gnt = 1 + rng.negative_binomial(GAS_TRK_NB[0], GAS_TRK_NB[1], n_gas)
        pz = np.concatenate([pz, gz])
        px = np.concatenate([px, gx])
        py = np.concatenate([py, gy])
        nt = np.concatenate([nt, gnt])
        gas = np.concatenate([gas, np.ones(n_gas, dtype=bool)])
    # interaction points follow the beamline: transverse offset + slope * z
    px = px + xb + txb * pz
    py = py + yb + tyb * pz
    n = int(nt.sum())
    pv_of = np.repeat(np.arange(nt.shape[0], dtype=np.int32), nt)
    tx = rng.normal(0.0, SLOPE_SIGMA, n)
    ty = rng.normal(0.0, SLOPE_SIGMA, n)
    displaced = rng.random(n) < DISPLACED_FRACTION
    flight = rng.exponential(DISPLACED_MEAN_LENGTH, n) * displaced
    norm = np.sqrt(1.0 + tx * tx + ty * ty)
    ox = px[pv_of] + flight * tx / norm
    oy = py[pv_of] + flight * ty / norm
    oz = pz[pv_of] + flight / norm
    sxy = rng.uniform(SIGMA_XY_RANGE[0], SIGMA_XY_RANGE[1], n)
    x = ox + sxy * rng.normal(0.0, 1.0, n)
    y = oy + sxy * rng.normal(0.0, 1.0, n)
    cov_xx = sxy * sxy
    if slope_cov:
        # a Kalman-like state covariance with slope terms (exercises Eq. 2):
        # sigma_t ~ U(2e-4, 2e-3), correlation rho ~ U(-0.6, 0.6)
        st = rng.uniform(2e-4, 2e-3, n)
        rho = rng.uniform(-0.6, 0.6, n)
        cov_xtx = rho * sxy * st
        cov_txtx = st * st
    else:
        cov_xtx = np.zeros(n)
        cov_txtx = np.zeros(n)
    perm = rng.permutation(n)
    cols = [a[perm] for a in (x, y, oz, tx, ty, cov_xx, cov_xtx, cov_txtx)]
    truth = np.stack([px, py, pz, gas.astype(np.float64)], axis=1)
    return cols, pv_of[perm], truth, nt


def generate(workload: str = "pp_mu5_100ev", n_events: Optional[int] = None, first_event: int = 0,
             beamline: Tuple[float, float, float, float] = (0.0, 0.0, 0.0, 0.0),
             slope_cov: bool = False, keep_truth: bool = True, **overrides) -> TrackBatch:
    """Generate events ``first_event .. first_event + n_events - 1`` of a workload.

    ``overrides`` may replace ``mu``, ``gas_mu``, ``config_id`` or
    ``mu_loguniform`` of the named workload.
    """
    spec = dict(WORKLOADS[workload])
    spec.update(overrides)
    if n_events is None:
        n_events = spec["n_events"]
    cfg = int(spec["config_id"])
    mu_lu = spec.get("mu_loguniform")
    cols_all: List[List[np.ndarray]] = [[] for _ in TRACK_FIELDS]
    counts = np.zeros(n_events, dtype=np.int64)
    truth_pvs, truth_nt, pv_of_all = [], [], []
    for i in range(n_events):
        ev = first_event + i
        rng = event_rng(cfg, ev)
        if mu_lu is not None:
            lo, hi = mu_lu
            mu = math.exp(rng.uniform(math.log(lo), math.log(hi)))
        else:
            mu = float(spec["mu"])
        cols, pv_of, truth, nt = _draw_event(rng, mu, float(spec.get("gas_mu", 0.0)), beamline, slope_cov)
        for k, c in enumerate(cols):
            cols_all[k].append(c)
        counts[i] = cols[0].shape[0]
        if keep_truth:
            truth_pvs.append(truth)
            truth_nt.append(nt)
            pv_of_all.append(pv_of)
    offs = np.zeros(n_events + 1, dtype=np.int64)
    offs[1:] = np.cumsum(counts)
    if offs[-1] >= 2 ** 31:
        raise ValueError("batch too large for int32 offsets")
    arrays = {f: (np.concatenate(cols_all[k]) if n_events else np.zeros(0)).astype(np.float32)
              for k, f in enumerate(TRACK_FIELDS)}
    return TrackBatch(offsets=offs.astype(np.int32), beamline=tuple(float(v) for v in beamline),
                      truth_pvs=truth_pvs if keep_truth else None,
                      truth_pv_of_track=(np.concatenate(pv_of_all).astype(np.int32)
                                         if keep_truth and n_events else None),
                      truth_ntracks=truth_nt if keep_truth else None, **arrays)


def _generate_chunk(args):
    workload, n, first, kw = args
    return generate(workload, n_events=n, first_event=first, keep_truth=False, **kw)


def generate_parallel(workload: str, n_events: Optional[int] = None, workers: int = 8,
                      chunk: int = 5000, **kw) -> TrackBatch:
    """``generate`` without truth, with chunks of events drawn in worker
    processes.  Every event has its own seed, so the batch is identical to
    ``generate(workload, n_events, keep_truth=False, **kw)``."""
    if n_events is None:
        n_events = WORKLOADS[workload]["n_events"]
    jobs = [(workload, min(chunk, n_events - a), a, kw) for a in range(0, n_events, chunk)]
    if workers <= 1 or len(jobs) <= 1:
        parts = [_generate_chunk(j) for j in jobs]
    else:
        import multiprocessing as mp
        with mp.get_context("spawn").Pool(min(workers, len(jobs))) as pool:
            parts = pool.map(_generate_chunk, jobs)
    return concat(parts) if parts else generate(workload, n_events=0, keep_truth=False, **kw)


def from_tracks(events: Sequence[np.ndarray], beamline=(0.0, 0.0, 0.0, 0.0)) -> TrackBatch:
    """Build a batch from explicit per-event (n, 8) arrays of track states
    (columns in TRACK_FIELDS order).  Used for hand-made edge cases."""
    mats = [np.asarray(e, dtype=np.float64).reshape(-1, 8) for e in events]
    counts = [m.shape[0] for m in mats]
    offs = np.zeros(len(mats) + 1, dtype=np.int32)
    offs[1:] = np.cumsum(counts)
    allm = np.concatenate(mats, axis=0) if mats else np.zeros((0, 8))
    arrays = {f: allm[:, k].astype(np.float32) for k, f in enumerate(TRACK_FIELDS)}
    return TrackBatch(offsets=offs, beamline=tuple(float(v) for v in beamline), **arrays)


def concat(batches: Sequence[TrackBatch]) -> TrackBatch:
    """Concatenate batches (same beamline) into one."""
    offs = [np.zeros(1, dtype=np.int64)]
    base = 0
    for b in batches:
        offs.append(b.offsets[1:].astype(np.int64) + base)
        base += b.n_tracks
    arrays = {f: np.concatenate([getattr(b, f) for b in batches]).astype(np.float32) for f in TRACK_FIELDS}
    return TrackBatch(offsets=np.concatenate(offs).astype(np.int32), beamline=batches[0].beamline, **arrays)
