"""Element-by-element comparison of the HIP path with the CPU oracle.

Bars (the same inputs on both sides):
* bit-exact: per-event status, histogram, per-track z_poca / sigma_poca /
  central bin (the binary32 stage), cluster bounds and peaks, association
  (kept flags, owned bins, track counts), vertex counts, per-track vertex ids;
* positions within POS_TOL_MM = 1e-3 mm and Tukey weights within
  W_TOL = 1e-4 (the targets stated for this path);
* seeds within SEED_TOL_MM: the GPU evaluates Eq. 4-5 in binary32, whose
  rounding near |z| = 600 mm is 3e-5 mm;
* covariance within COV_RTOL relative to its largest element, chi2 / ndof
  within CHI2_TOL_PER_TRACK per track: both are sums over tracks of
  quantities whose weights agree to W_TOL.
A convergence decision the oracle took within TIE_MARGIN (relative) of its
threshold may go the other way in binary32; such a vertex is a reported tie:
its iteration count and weights are not compared, its position must still
agree within TIE_POS_TOL_MM (one more or one less step moves it by less than
the 1 micrometre convergence threshold).

Multi-vertex variant (Eq. 18): the pre-cut is binary32 on both sides, so the
candidates' list lengths are compared bit-exactly.  Three decisions follow a
binary32 fit on the GPU and a binary64 fit in the oracle, and count as ties
when the oracle took them within a margin: a vertex's track count may differ
by the tracks whose oracle weight lies within 1e-4 of w_count_mv; an event's
vertex count may differ when one of its vertices had such tracks or a
duplicate test within 1 % of its threshold; a track may report another vertex
when its weight there equals the oracle's best within W_TOL.
"""
import dataclasses
from typing import Dict, List

import numpy as np

import oracle
from paper_2412_14966_amd import pvfind as pv

POS_TOL_MM = 1e-3
W_TOL = 1e-4
SEED_TOL_MM = 1e-4
COV_RTOL = 2e-3
CHI2_TOL_PER_TRACK = 2e-3
TIE_MARGIN = 2e-2
TIE_POS_TOL_MM = 2e-3


def oracle_params(lib_params: pv.pv_params) -> Dict:
    """The oracle's parameter set holding exactly the library's values."""
    return oracle.params_from_fields(pv.params_dict(lib_params))


@dataclasses.dataclass
class Report:
    n_events: int = 0
    n_vertices: int = 0
    n_tracks: int = 0
    ties: int = 0
    max_dpos: float = 0.0
    max_dw: float = 0.0
    max_dseed: float = 0.0
    max_dcov: float = 0.0
    max_dchi2: float = 0.0
    fp64_inversions: int = 0
    problems: List[str] = dataclasses.field(default_factory=list)

    def fail(self, msg):
        if len(self.problems) < 40:
            self.problems.append(msg)

    def ok(self):
        return not self.problems

    def summary(self):
        return (f"events={self.n_events} vertices={self.n_vertices} tracks={self.n_tracks} ties={self.ties} "
                f"max|dpos|={self.max_dpos:.3g} max|dw|={self.max_dw:.3g} max|dseed|={self.max_dseed:.3g} "
                f"max cov rel={self.max_dcov:.3g} max|dchi2|/trk={self.max_dchi2:.3g} "
                f"fp64_inv={self.fp64_inversions} problems={len(self.problems)}")


def _f32_bits(a):
    return np.ascontiguousarray(a, dtype=np.float32).view(np.uint32)


def compare(batch, g: "pv.HostResult", o: "oracle.OracleResult", debug: bool = False,
            fit: bool = True, mv: bool = False) -> Report:
    """Compare everything; with fit=False only the stages defined bit-exactly
    (status, binary32 projection, histogram, clusters, association)."""
    r = Report(n_events=batch.n_events, n_tracks=batch.n_tracks)
    if not np.array_equal(g.status, o.status):
        bad = np.nonzero(g.status != o.status)[0][:5]
        r.fail(f"status differs at events {bad.tolist()}: gpu {g.status[bad].tolist()} oracle {o.status[bad].tolist()}")
    valid_ev = (o.status & oracle.EV_OFFSETS_INVALID) == 0
    if debug:
        if not np.array_equal(g.hist, o.hist):
            bad = np.nonzero(np.any(g.hist != o.hist, axis=1))[0][:5]
            r.fail(f"histogram differs in events {bad.tolist()}")
        in_ev = np.zeros(batch.n_tracks, dtype=bool)
        for e in np.nonzero(valid_ev)[0]:
            in_ev[batch.offsets[e]:batch.offsets[e + 1]] = True
        too_many = np.zeros(batch.n_tracks, dtype=bool)
        for e in np.nonzero(o.status & oracle.EV_TOO_MANY_TRACKS)[0]:
            too_many[batch.offsets[e]:batch.offsets[e + 1]] = True
        sel = in_ev & ~too_many
        for name in ("zpoca", "sigma"):
            gb, ob = _f32_bits(getattr(g, name))[sel], _f32_bits(getattr(o, name))[sel]
            if not np.array_equal(gb, ob):
                k = np.nonzero(gb != ob)[0][:5]
                r.fail(f"{name} bits differ at tracks {k.tolist()}")
        if not np.array_equal(g.bin[sel], o.bin[sel]):
            r.fail("central bins differ")
        if not np.array_equal(g.n_clusters, o.n_clusters):
            bad = np.nonzero(g.n_clusters != o.n_clusters)[0][:5]
            r.fail(f"cluster counts differ at events {bad.tolist()}")
        else:
            for e in range(batch.n_events):
                n = int(o.n_clusters[e])
                gc, oc = g.clusters[e, :n], o.clusters[e, :n]
                for f in ("lo", "hi", "peak", "kept", "n_assoc"):
                    if not np.array_equal(gc[f], oc[f]):
                        r.fail(f"event {e}: cluster field {f} differs")
                kept = oc["kept"] == 1
                for f in ("own_lo", "own_hi"):
                    if not np.array_equal(gc[f][kept], oc[f][kept]):
                        r.fail(f"event {e}: cluster field {f} differs")
                if n:
                    d = float(np.max(np.abs(gc["z_seed"].astype(np.float64) - oc["z_seed"])))
                    r.max_dseed = max(r.max_dseed, d)
                    if d > SEED_TOL_MM:
                        r.fail(f"event {e}: seed z differs by {d}")

    if not fit:
        return r
    tie_tracks = np.zeros(batch.n_tracks, dtype=bool)
    for e in range(batch.n_events):
        if not valid_ev[e]:
            continue
        ng, no = int(g.n_vertices[e]), int(o.n_vertices[e])
        if ng != no:
            ovs = o.vertices[e, :no]
            if mv and no and (np.any(ovs["n_near"] > 0) or np.any(ovs["dup_margin"] < 1e-2)):
                r.ties += 1
            else:
                r.fail(f"event {e}: {ng} vertices on the GPU, {no} in the oracle")
            continue
        r.n_vertices += no
        gv, ov = g.vertices[e, :no], o.vertices[e, :no]
        a, b = batch.offsets[e], batch.offsets[e + 1]
        for k in range(no):
            for f, of in (("bin_lo", "bin_lo"), ("bin_hi", "bin_hi"), ("peak_bin", "peak_bin"),
                          ("n_tracks", "n_tracks")):
                d = abs(int(gv[k][f]) - int(ov[k][of]))
                allowed = int(ov[k]["n_near"]) if (mv and f == "n_tracks") else 0
                if d > allowed:
                    r.fail(f"event {e} vertex {k}: {f} {int(gv[k][f])} vs {int(ov[k][of])}")
                elif d:
                    r.ties += 1
            tie = int(gv[k]["n_iter"]) != int(ov[k]["n_iter"])
            if tie:
                if ov[k]["conv_margin"] < TIE_MARGIN:
                    r.ties += 1
                    tie_tracks[a:b] |= (o.track_vertex[a:b] == k)
                else:
                    r.fail(f"event {e} vertex {k}: n_iter {int(gv[k]['n_iter'])} vs {int(ov[k]['n_iter'])} "
                           f"(margin {ov[k]['conv_margin']:.3g})")
            dpos = max(abs(float(gv[k][c]) - float(ov[k][c])) for c in ("x", "y", "z"))
            r.max_dpos = max(r.max_dpos, dpos)
            if dpos > (TIE_POS_TOL_MM if tie else POS_TOL_MM):
                r.fail(f"event {e} vertex {k}: position differs by {dpos:.3g} mm")
            if not tie:
                gnc = bool(gv[k]["flags"] & pv.PV_VX_NOT_CONVERGED)
                onc = bool(ov[k]["flags"] & oracle.VX_NOT_CONVERGED)
                if gnc != onc:
                    r.fail(f"event {e} vertex {k}: convergence flag differs")
                cg = np.asarray(gv[k]["cov"], dtype=np.float64)
                co = np.asarray(ov[k]["cov"], dtype=np.float64)
                rel = float(np.max(np.abs(cg - co)) / max(np.max(np.abs(co)), 1e-300))
                r.max_dcov = max(r.max_dcov, rel)
                if rel > COV_RTOL:
                    r.fail(f"event {e} vertex {k}: covariance differs by {rel:.3g} (relative)")
                nt = max(int(ov[k]["n_tracks"]), 1)
                dchi = max(abs(float(gv[k]["chi2"]) - float(ov[k]["chi2"])),
                           abs(float(gv[k]["ndof"]) - float(ov[k]["ndof"]))) / nt
                r.max_dchi2 = max(r.max_dchi2, dchi)
                if dchi > CHI2_TOL_PER_TRACK:
                    r.fail(f"event {e} vertex {k}: chi2/ndof differ by {dchi:.3g} per track")
            if gv[k]["flags"] & pv.PV_VX_FP64_INVERSION:
                r.fp64_inversions += 1

    # per-track outputs of valid events
    sel = np.zeros(batch.n_tracks, dtype=bool)
    for e in np.nonzero(valid_ev)[0]:
        if g.n_vertices[e] == o.n_vertices[e]:
            sel[batch.offsets[e]:batch.offsets[e + 1]] = True
    diff = (g.track_vertex != o.track_vertex) & sel
    if mv and np.any(diff):
        # another vertex of (within tolerance) the same, largest weight
        same = diff & (np.abs(g.track_weight.astype(np.float64) - o.track_weight) < W_TOL) & \
            (g.track_vertex >= 0) & (o.track_vertex >= 0)
        r.ties += int(np.sum(same))
        tie_tracks |= same
        diff &= ~same
    if np.any(diff):
        k = np.nonzero(diff)[0][:5]
        r.fail(f"track vertex ids differ at tracks {k.tolist()}")
    cmp = sel & ~tie_tracks
    if np.any(cmp):
        dw = np.abs(g.track_weight[cmp].astype(np.float64) - o.track_weight[cmp])
        r.max_dw = float(dw.max())
        if r.max_dw > W_TOL:
            k = np.nonzero(cmp)[0][np.argmax(dw)]
            r.fail(f"track weight differs by {r.max_dw:.3g} at track {int(k)}")
    return r
