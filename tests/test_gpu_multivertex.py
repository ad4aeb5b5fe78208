"""GPU parity of the multi-vertex variant (Sec. 3.5 and Sec. 5: every track
weighted to every candidate with Eq. 18, chi2 pre-cut, |dz| convergence,
duplicate rejection) against the oracle's same variant.  The pre-cut is
binary32 on both sides and compared bit-exactly (candidate list lengths);
decisions after the binary32 fit follow the tie rules of tests/parity.py."""
import sys

import numpy as np
import pytest

import oracle
import parity
from paper_2412_14966_amd import pvfind as pv, synth
from test_gpu_parity import _exact_event, _spread_event

pytestmark = pytest.mark.gpu

MV = {"assoc_mode": 1}


def say(msg):
    print(f"[gpu-mv] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pv.lib()
    yield


def check(batch, params=None, schedule=None, debug=True, name="", max_tie_frac=0.01):
    prm = dict(MV, **(params or {}))
    p = pv.make_params(prm)
    say(f"{name}: {batch.n_events} events, {batch.n_tracks} tracks, schedule={schedule}, debug={debug}")
    g = pv.run(batch, prm, schedule=schedule, debug=debug)
    o = oracle.find(batch, parity.oracle_params(p), debug=debug)
    rep = parity.compare(batch, g, o, debug=debug, mv=True)
    say(f"{name}: {rep.summary()}")
    assert rep.ok(), "\n".join(rep.problems)
    assert rep.ties <= max(3, max_tie_frac * rep.n_vertices)
    return g, o, rep


def test_mv_config1_debug():
    check(synth.generate("pp_mu5_100ev"), name="mv pp mu=5 100 events")


def test_mv_full_size_bench_workload():
    """10,000 events at mu = 5 in the benchmark's launch configuration."""
    check(synth.generate("pp_mu5_10kev", keep_truth=False), debug=False, name="mv pp mu=5 10k events")


def test_mv_beam_gas_and_high_pileup_samples():
    check(synth.generate("pp_mu5_gas_50kev", n_events=3000, keep_truth=False), name="mv pp + beam-gas 3k")
    check(synth.generate("pp_mu40_20kev", n_events=400, keep_truth=False), name="mv mu=40 400 events")


@pytest.mark.parametrize("sched", [dict(waves_per_team=w, track_capacity=c, persistent=m, teams_per_cu=0)
                                   for (w, c, m) in ((1, 256, 2), (2, 512, 4), (4, 1024, 2), (2, 1024, 4))],
                         ids=lambda s: f"w{s['waves_per_team']}c{s['track_capacity']}m{s['persistent']}")
def test_mv_schedules_and_deferrals(sched):
    """Small teams hand the large-event launch the events whose tracks,
    touched words, clusters or candidate lists exceed them: a 700-track
    vertex, 34 vertices packed at the low end, 72 gas clusters."""
    rng = np.random.default_rng(44)
    evs = [_spread_event(np.linspace(-500, 300, 20), 6, rng),
           _spread_event(-590.0 + 6.0 * np.arange(34), 5, rng),
           _spread_event(-598.0 + 4.0 * np.arange(72), 4, rng),
           _exact_event((0.0, 0.0, 5.0), 700, rng)]
    b = synth.concat([synth.generate("pp_mu5_100ev", n_events=30), synth.from_tracks(evs)])
    check(b, schedule=sched, name="mv schedules")


@pytest.mark.parametrize("sched", [dict(waves_per_team=w, track_capacity=c, persistent=m, teams_per_cu=0)
                                   for (w, c, m) in ((4, 1536, 4), (1, 1024, 2), (2, 2048, 4), (8, 1536, 4))],
                         ids=lambda s: f"w{s['waves_per_team']}c{s['track_capacity']}m{s['persistent']}")
def test_mv_high_pileup_precut_in_z_order(sched):
    """At mu = 40 (~35 candidates) small teams take the pre-cut's tracks in z
    order and try only the candidates within reach of each chunk: the lists,
    and so every output, still match the oracle, for one, two and four
    wavefronts per team and eight (the high pile-up schedule among them)."""
    b = synth.generate("pp_mu40_20kev", n_events=300, keep_truth=False)
    g, o, rep = check(b, schedule=sched, debug=False, name=f"mv mu=40 z order {sched}")
    assert rep.n_vertices > 300 * 25   # ~34 vertices per event: the z-ordered path runs


def test_mv_candidate_lists_beyond_the_track_limit():
    """An unbounded pre-cut puts every track in every candidate's list: events
    whose lists exceed max_tracks_per_event are flagged and give no vertex,
    the others still match the oracle."""
    b = synth.generate("pp_mu5_100ev", n_events=40)
    g, o, rep = check(b, {"chi2_window_mv": 1e30, "max_tracks_per_event": 1024}, name="mv lists over the limit")
    assert np.any(o.status & oracle.EV_TOO_MANY_TRACKS)
    assert np.any((o.status & oracle.EV_TOO_MANY_TRACKS) == 0)


def test_mv_duplicates_and_open_selection():
    """Duplicate rejection with a large ratio drops many candidates; with the
    selection opened up every surviving fit is written."""
    b = synth.generate("pp_mu40_20kev", n_events=100, keep_truth=False)
    check(b, {"dup_ratio": 400.0}, name="mv duplicates R=400")
    check(b, {"pv_min_pp": 0, "pv_min_gas": 0, "max_rho_pp": 1e9, "dup_ratio": 0.0}, name="mv open selection")


def test_mv_duplicates_in_large_event_teams():
    """Events of ~100 interactions (2,300-3,100 tracks, 68-81 vertices) go to
    the large-event teams, whose 128 candidate slots take two per lane in the
    duplicate test; a ratio of 10^4 makes long chains of duplicates (40-48
    vertices kept), decided in rank order."""
    b = synth.generate("pp_mu40_20kev", n_events=6, mu=100.0, keep_truth=False)
    g, o, rep = check(b, name="mv large events, default ratio")
    assert int(np.max(o.n_vertices)) > 64
    g, o, rep = check(b, {"dup_ratio": 1e4}, name="mv duplicates, large events, R=1e4")
    assert int(np.max(o.n_vertices)) < 50


def test_mv_empty_and_tiny_events():
    """Alternating empty events, one to three tracks and mu = 5 events, over
    two ordering slices."""
    rng = np.random.default_rng(35)
    real = synth.generate("pp_mu5_10kev", n_events=400, keep_truth=False)
    evs = []
    for k in range(1100):
        if k % 3 == 0:
            evs.append(np.zeros((0, 8)))
        elif k % 3 == 1:
            t = np.zeros((int(rng.integers(1, 4)), 8))
            t[:, 2] = rng.uniform(-50, 50, len(t))
            t[:, 3:5] = rng.normal(0, 0.2, (len(t), 2))
            t[:, 5] = 1e-3
            evs.append(t)
        else:
            e = (k // 3) % real.n_events
            a, z = int(real.offsets[e]), int(real.offsets[e + 1])
            evs.append(np.stack([getattr(real, f)[a:z] for f in synth.TRACK_FIELDS], axis=1))
    g, o, rep = check(synth.from_tracks(evs), name="mv empty/tiny/mu5 events")
    assert np.all(g.n_vertices[0::3] == 0)


def test_mv_tilted_offset_beamline_and_slope_covariance():
    """Kalman-like covariances with slope terms (Eq. 2 at the seed) and a
    displaced, tilted beamline."""
    b = synth.generate("pp_mu5_100ev", beamline=(1.092, 0.472, 2e-4, -1e-4), slope_cov=True)
    check(b, name="mv offset tilted beamline, slope covariance")
    check(b, {"peak_mode": 1}, name="mv + recursive splitting, offset tilted beamline")
