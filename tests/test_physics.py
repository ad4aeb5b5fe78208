"""The Sec. 4 figures of merit (paper_2412_14966_amd/physics.py) on hand-made
truth and on the oracle's reconstruction of synthetic events."""
import numpy as np
import pytest

import oracle
from paper_2412_14966_amd import physics, synth


def _rec(zs, czz, ntr=None):
    r = np.zeros(len(zs), dtype=[("x", "f8"), ("y", "f8"), ("z", "f8"), ("cov", "f8", (6,)), ("n_tracks", "i4")])
    r["z"] = zs
    r["cov"][:, 0] = r["cov"][:, 2] = 1e-4
    r["cov"][:, 5] = czz
    r["n_tracks"] = ntr if ntr is not None else 20
    return r


def test_matching_rules_by_hand():
    """Reconstructible: >= 4 tracks pp, >= 3 p-gas.  Matched within 5 sigma_z
    to the closest reconstructible PV; of two matches of one PV only the
    closer counts; a match outside 5 sigma is a fake."""
    true = np.array([[0, 0, 0.0, 0], [0, 0, 30.0, 0], [0, 0, 60.0, 0], [0, 0, -400.0, 1]])
    ntr = np.array([30, 3, 12, 3])          # the 3-track pp PV is not reconstructible, the gas one is
    rec = _rec([0.02, 0.05, 30.0, 60.3, -400.1], [1e-4, 1e-4, 1e-4, 1e-2, 1e-2])
    rcible, match = physics.match_event(true, ntr, rec)
    assert rcible.tolist() == [True, False, True, True]
    # 0.02 and 0.05 both within 5 sigma (0.05 mm) of z = 0: the closer keeps it;
    # 30.0 has no reconstructible partner; 60.3 is 3 sigma from 60; -400.1 is 1 sigma from -400
    assert match.tolist() == [0, -1, -1, 2, 3]

    class B:
        n_events = 1
        truth_pvs = [true]
        truth_ntracks = [ntr]
    res = physics.evaluate(B, np.array([5]), rec.reshape(1, -1))
    assert res["reconstructible"] == 3 and res["matched"] == 3
    assert res["efficiency"] == 1.0 and res["fake_rate"] == pytest.approx(2 / 5)
    assert res["efficiency_isolated"] == 1.0 and np.isnan(res["efficiency_close"])


def test_close_and_rank_categories_by_hand():
    true = np.array([[0, 0, 0.0, 0], [0, 0, 5.0, 0], [0, 0, 50.0, 0]])
    ntr = np.array([10, 40, 20])
    rec = _rec([5.0, 50.0], [1e-4, 1e-4])

    class B:
        n_events = 1
        truth_pvs = [true]
        truth_ntracks = [ntr]
    res = physics.evaluate(B, np.array([2]), rec.reshape(1, -1))
    assert res["efficiency_close"] == pytest.approx(0.5)       # the PVs at 0 and 5 mm are close
    assert res["efficiency_isolated"] == 1.0
    assert res["efficiency_by_rank"][:3] == [1.0, 1.0, 0.0]     # 40, 20, 10 tracks


def _oracle_rec(batch, params=None):
    o = oracle.find(batch, params)
    return o.n_vertices, o.vertices


def test_oracle_reconstruction_is_self_consistent():
    """On synthetic mu = 5 events the reconstruction finds most PVs, few fakes,
    and its uncertainties describe its errors (pulls of width near one)."""
    b = synth.generate("pp_mu5_100ev", n_events=400)
    res = physics.evaluate(b, *_oracle_rec(b))
    assert res["efficiency"] > 0.85 and res["fake_rate"] < 0.1
    assert res["efficiency_by_rank"][0] > 0.97
    for c in "xyz":
        assert 0.6 < res["pull_width"][c] < 1.6 and abs(res["pull_mean"][c]) < 0.3
    mv = physics.evaluate(b, *_oracle_rec(b, {"assoc_mode": 1}))
    assert mv["efficiency"] > 0.85 and mv["fake_rate"] < 0.1


def test_beamline_offset_robustness():
    """A transverse beamline error of 20 um barely changes the efficiency
    (the paper: 99.9 % of it within 20 um, 99 % within 50 um)."""
    b = synth.generate("pp_mu5_100ev", n_events=300)
    base = physics.evaluate(b, *_oracle_rec(b))["efficiency"]
    shifted = synth.TrackBatch(offsets=b.offsets, beamline=(0.02, 0.02, 0.0, 0.0), truth_pvs=b.truth_pvs,
                               truth_ntracks=b.truth_ntracks, **{f: getattr(b, f) for f in synth.TRACK_FIELDS})
    eff = physics.evaluate(shifted, *_oracle_rec(shifted))["efficiency"]
    assert eff / base > 0.98
