"""The bound behind the multi-vertex pre-cut's z windows (the kernels skip a
candidate for a chunk of tracks when its seed lies outside every track's
window): a track whose z_poca (Eq. 1) is farther than
A = s (sigma_x + |z_poca - z| sigma_tx) / (|dt| - s sigma_tx), s = sqrt(cut),
from a seed on the beamline has chi2 >= cut at that seed, with chi2 from
Eq. 7 and Eq. 9 and V_x from Eq. 2 at the seed.  Checked in binary64 on
every (track, candidate) pair of high pile-up events, with covariances that
include slope terms, against the seeds the oracle finds."""
import numpy as np
import pytest

import oracle
from paper_2412_14966_amd import synth


def _pairs(batch, res):
    for e in range(batch.n_events):
        a0, a1 = batch.offsets[e], batch.offsets[e + 1]
        sl = slice(a0, a1)
        t = [np.asarray(getattr(batch, f)[sl], dtype=np.float64) for f in synth.TRACK_FIELDS]
        zs = res.clusters[e, :res.n_clusters[e]]["z_seed"]
        yield t, zs, res.bin[sl] >= 0


def _transported(b, dz):
    """The same tracks with their states (and covariances, as Eq. 2) given
    dz further along z."""
    f = {k: np.asarray(getattr(b, k), dtype=np.float64) for k in synth.TRACK_FIELDS}
    g = dict(x=f["x"] + f["tx"] * dz, y=f["y"] + f["ty"] * dz, z=f["z"] + dz, tx=f["tx"], ty=f["ty"],
             cov_xx=f["cov_xx"] + 2.0 * dz * f["cov_xtx"] + dz * dz * f["cov_txtx"],
             cov_xtx=f["cov_xtx"] + dz * f["cov_txtx"], cov_txtx=f["cov_txtx"])
    return synth.TrackBatch(offsets=b.offsets, beamline=b.beamline,
                            **{k: v.astype(np.float32) for k, v in g.items()})


@pytest.mark.parametrize("dz", [0.0, 250.0])
def test_tracks_outside_their_window_fail_the_precut(dz):
    cut = 25.0
    b = synth.generate("pp_mu40_20kev", n_events=60, keep_truth=False, slope_cov=True)
    if dz:
        b = _transported(b, dz)   # states far from z_poca: the sigma_tx terms matter
    bx, by, btx, bty = (float(v) for v in b.beamline)
    r = oracle.find(b, {"assoc_mode": 1}, debug=True)
    outside = inside = 0
    for (x, y, z, tx, ty, vxx, vxtx, vtxtx), zs, assoc in _pairs(b, r):
        dtx, dty = tx - btx, ty - bty
        den = dtx * dtx + dty * dty
        zp = z + (dtx * (bx - x) + dty * (by - y)) / den
        psd = vxtx * vxtx <= vxx * vtxtx
        s = np.sqrt(cut)
        g = np.sqrt(den) - s * np.sqrt(vtxtx)
        A = np.where(psd & (g > 0), s * (np.sqrt(vxx) + np.abs(zp - z) * np.sqrt(vtxtx)) / np.where(g > 0, g, 1.0),
                     np.inf)
        # chi2 at every seed (Eq. 9 residual, Eq. 2 variance, Eq. 7)
        Z = zs[None, :]
        rx = x[:, None] + tx[:, None] * (Z - z[:, None]) - (bx + btx * Z)
        ry = y[:, None] + ty[:, None] * (Z - z[:, None]) - (by + bty * Z)
        d = Z - z[:, None]
        V = vxx[:, None] + 2.0 * d * vxtx[:, None] + d * d * vtxtx[:, None]
        chi2 = (rx * rx + ry * ry) / V
        far = (np.abs(Z - zp[:, None]) > A[:, None]) & assoc[:, None]
        assert np.all(chi2[far] >= cut), chi2[far].min()
        outside += int(far.sum())
        inside += int((~far & assoc[:, None]).sum())
    # the windows leave out most pairs at this pile-up (the kernels' saving)
    assert outside > 5 * inside, (outside, inside)
