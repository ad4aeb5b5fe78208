"""Figures of merit of the paper's physics study (Sec. 4) on generator truth.

The paper measures efficiency, fake rate, position resolution and pull on
LHCb simulation; here the same definitions are applied to the synthetic
events of ``synth`` (whose truth is their generator's), as a self-consistency
check of the reconstruction, not a reproduction of the paper's numbers.

Definitions (Sec. 4):
* a simulated PV is reconstructible with at least 4 tracks (3 for p-gas);
* a reconstructed PV matches a reconstructible simulated PV when their z
  differ by less than five times the reconstructed z uncertainty; it is
  matched to the closest such PV, and a simulated PV matched by several
  reconstructed PVs keeps only the closest;
* efficiency = matched / reconstructible; fake rate = (reconstructed -
  matched) / reconstructed;
* resolution = standard deviation of (reconstructed - simulated) per
  coordinate over matched pairs; pull = that difference over the
  reconstructed uncertainty (mean and standard deviation);
* categories: ``close`` when another reconstructible PV of the event lies
  within 10 mm in z, else ``isolated``; multiplicity rank within the event
  (1st = most tracks).

``python -m paper_2412_14966_amd.physics --workload pp_mu5_100ev --events 2000``
runs the HIP library on a workload and prints the figures, and with
``--beam-offsets`` the efficiency when the beamline given to the algorithm
is displaced from the generated one (the paper's robustness study).
"""
from __future__ import annotations

import argparse
import json
import sys
from typing import Dict, Optional, Sequence

import numpy as np

CLOSE_MM = 10.0
N_SIGMA = 5.0


def match_event(true_pvs: np.ndarray, true_ntracks: np.ndarray, rec: np.ndarray,
                min_pp: int = 4, min_gas: int = 3, n_sigma: float = N_SIGMA):
    """Reconstructible flags of the simulated PVs and, per reconstructed PV,
    the index of its matched simulated PV (-1 if none).  rec holds records
    with fields z and cov (cov[5] = C_zz)."""
    gas = true_pvs[:, 3] > 0.5 if true_pvs.shape[0] else np.zeros(0, bool)
    rcible = true_ntracks >= np.where(gas, min_gas, min_pp)
    match = np.full(rec.shape[0], -1, dtype=np.int64)
    dist = np.full(rec.shape[0], np.inf)
    cand = np.nonzero(rcible)[0]
    for r in range(rec.shape[0]):
        sz = float(np.sqrt(max(float(rec[r]["cov"][5]), 0.0)))
        if cand.size == 0:
            continue
        d = np.abs(true_pvs[cand, 2] - float(rec[r]["z"]))
        k = int(np.argmin(d))
        if d[k] < n_sigma * sz:
            match[r] = int(cand[k])
            dist[r] = float(d[k])
    # a simulated PV keeps only its closest reconstructed match
    for t in np.unique(match[match >= 0]):
        rs = np.nonzero(match == t)[0]
        keep = rs[np.argmin(dist[rs])]
        match[rs[rs != keep]] = -1
    return rcible, match


def evaluate(batch, n_vertices: np.ndarray, vertices: np.ndarray, min_pp: int = 4, min_gas: int = 3,
             n_sigma: float = N_SIGMA, max_rank: int = 5) -> Dict:
    """Figures of merit over a batch with truth.  vertices: (n_events,
    max_vertices) records with x, y, z, cov and n_tracks."""
    if batch.truth_pvs is None:
        raise ValueError("the batch carries no truth (generate it with keep_truth=True)")
    n_rcible = n_matched = n_rec = n_rec_matched = 0
    n_rec10 = n_rec10_matched = 0
    cat = {"isolated": [0, 0], "close": [0, 0]}
    rank = [[0, 0] for _ in range(max_rank)]
    diffs, pulls = [], []
    for e in range(batch.n_events):
        tp = np.asarray(batch.truth_pvs[e], dtype=np.float64).reshape(-1, 4)
        tn = np.asarray(batch.truth_ntracks[e])
        rec = vertices[e, :int(n_vertices[e])]
        rcible, match = match_event(tp, tn, rec, min_pp, min_gas, n_sigma)
        found = np.zeros(tp.shape[0], dtype=bool)
        found[match[match >= 0]] = True
        n_rcible += int(rcible.sum())
        n_matched += int(found.sum())
        n_rec += rec.shape[0]
        n_rec_matched += int(np.sum(match >= 0))
        big = rec["n_tracks"] >= 10
        n_rec10 += int(big.sum())
        n_rec10_matched += int(np.sum(big & (match >= 0)))
        idx = np.nonzero(rcible)[0]
        for t in idx:
            others = idx[idx != t]
            close = bool(others.size and np.min(np.abs(tp[others, 2] - tp[t, 2])) < CLOSE_MM)
            c = cat["close" if close else "isolated"]
            c[0] += 1
            c[1] += int(found[t])
        order = idx[np.argsort(-tn[idx], kind="stable")]
        for k, t in enumerate(order[:max_rank]):
            rank[k][0] += 1
            rank[k][1] += int(found[t])
        for r in np.nonzero(match >= 0)[0]:
            t = match[r]
            d = np.array([float(rec[r]["x"]) - tp[t, 0], float(rec[r]["y"]) - tp[t, 1], float(rec[r]["z"]) - tp[t, 2]])
            s = np.sqrt(np.maximum(np.array([rec[r]["cov"][0], rec[r]["cov"][2], rec[r]["cov"][5]], dtype=np.float64),
                                   1e-300))
            diffs.append(d)
            pulls.append(d / s)
    diffs = np.array(diffs).reshape(-1, 3)
    pulls = np.array(pulls).reshape(-1, 3)

    def frac(a, b):
        return float(a) / float(b) if b else float("nan")

    out = {
        "events": batch.n_events,
        "reconstructible": n_rcible, "reconstructed": n_rec, "matched": n_rec_matched,
        "efficiency": frac(n_matched, n_rcible),
        "fake_rate": frac(n_rec - n_rec_matched, n_rec),
        "fake_rate_ge10_tracks": frac(n_rec10 - n_rec10_matched, n_rec10),
        "efficiency_isolated": frac(cat["isolated"][1], cat["isolated"][0]),
        "efficiency_close": frac(cat["close"][1], cat["close"][0]),
        "efficiency_by_rank": [frac(f, n) for n, f in rank],
    }
    if diffs.shape[0] > 1:
        out["resolution_mm"] = dict(zip("xyz", np.std(diffs, axis=0, ddof=1).tolist()))
        out["pull_mean"] = dict(zip("xyz", np.mean(pulls, axis=0).tolist()))
        out["pull_width"] = dict(zip("xyz", np.std(pulls, axis=0, ddof=1).tolist()))
    return out


def _run_gpu(batch, params: Optional[Dict], beamline: Sequence[float]):
    from . import pvfind as pv, synth
    b = synth.TrackBatch(offsets=batch.offsets, beamline=tuple(float(v) for v in beamline),
                         **{f: getattr(batch, f) for f in synth.TRACK_FIELDS})
    r = pv.run(b, params)
    return r.n_vertices, r.vertices


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("--workload", default="pp_mu5_100ev")
    ap.add_argument("--events", type=int, default=2000)
    ap.add_argument("--multivertex", action="store_true", help="the GPU-variant association (Eq. 18)")
    ap.add_argument("--beam-offsets", default="", help="comma-separated transverse beamline offsets in mm")
    a = ap.parse_args(argv)
    from . import synth
    batch = synth.generate(a.workload, n_events=a.events)
    params = {"assoc_mode": 1} if a.multivertex else None
    nv, vx = _run_gpu(batch, params, batch.beamline)
    res = evaluate(batch, nv, vx)
    if a.beam_offsets:
        base = res["efficiency"]
        res["relative_efficiency_vs_beam_offset_mm"] = {}
        for off in (float(v) for v in a.beam_offsets.split(",")):
            bl = list(batch.beamline)
            bl[0] += off
            bl[1] += off
            nv2, vx2 = _run_gpu(batch, params, bl)
            res["relative_efficiency_vs_beam_offset_mm"][str(off)] = evaluate(batch, nv2, vx2)["efficiency"] / base
    json.dump(res, sys.stdout, indent=1)
    print()
    return 0


if __name__ == "__main__":
    sys.exit(main())
