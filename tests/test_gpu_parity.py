"""Parity of the HIP path with the CPU oracle on the GPU (bars in parity.py).

Every call goes through the C ABI (paper_2412_14966_amd.pvfind -> libpvfind).
"""
import sys

import numpy as np
import pytest

import oracle
from paper_2412_14966_amd import pvfind as pv
from paper_2412_14966_amd import synth

import parity

pytestmark = pytest.mark.gpu

SCHEDULES = [dict(waves_per_team=w, track_capacity=c, persistent=m, teams_per_cu=0)
             for w in (1, 2, 4, 8) for c in (256, 512, 1024, 1536, 2048) for m in (2, 4)
             if not (w == 8 and c < 1024)]
WAVE = [dict(waves_per_team=1, track_capacity=c, persistent=m, teams_per_cu=0) for c in (256, 512) for m in (1, 2)]
TEAM = dict(waves_per_team=2, track_capacity=512, persistent=2, teams_per_cu=0)


def say(msg):
    print(f"[gpu] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pv.lib()
    yield


def run_both(batch, params=None, schedule=None, debug=True, name=""):
    p = pv.make_params(params)
    say(f"{name}: {batch.n_events} events, {batch.n_tracks} tracks, schedule={schedule}, debug={debug}")
    g = pv.run(batch, params, schedule=schedule, debug=debug)
    o = oracle.find(batch, parity.oracle_params(p), debug=debug)
    return g, o


def check(batch, params=None, schedule=None, debug=True, name="", max_tie_frac=0.01, fit=True):
    g, o = run_both(batch, params, schedule, debug, name)
    rep = parity.compare(batch, g, o, debug=debug, fit=fit)
    say(f"{name}: {rep.summary()}")
    assert rep.ok(), "\n".join(rep.problems)
    assert rep.ties <= max(2, max_tie_frac * rep.n_vertices)
    return g, o, rep


def test_projection_bit_exact_on_a_million_tracks():
    """Random tracks (slopes down to 1e-3, not from vertices): the binary32
    projection, the histogram, clusters and association must be bit-exact.
    Their 'vertices' are fits of unrelated tracks with normal matrices of
    condition ~1e6, which a binary32 fit does not follow; the fit is compared
    on the physical workloads below."""
    rng = np.random.default_rng(20)
    n = 1 << 20
    cols = np.zeros((n, 8))
    cols[:, 0:2] = rng.normal(0, 0.1, (n, 2))
    cols[:, 2] = rng.uniform(-650, 450, n)
    cols[:, 3:5] = rng.normal(0, 0.3, (n, 2)) * rng.choice([1e-3, 1e-2, 1.0, 3.0], (n, 1))
    cols[:, 5] = rng.uniform(1e-5, 3e-3, n)
    # 1024 events of 1024 tracks
    b = synth.from_tracks(np.split(cols, 1024), beamline=(0.01, -0.02, 1e-4, -2e-4))
    check(b, {"max_tracks_per_event": 1024}, name="projection 1M", fit=False)


def test_config1_full_parity_debug():
    b = synth.generate("pp_mu5_100ev")
    check(b, name="pp mu=5 100 events")


def test_config1_tilted_offset_beamline_and_slope_covariance():
    b = synth.generate("pp_mu5_100ev", beamline=(1.092, 0.472, 2e-4, -1e-4), slope_cov=True)
    check(b, name="offset tilted beamline, slope covariance")


def _exact_event(P, n, rng, slopes=None, var=2.0 ** -11):
    rows = []
    for k in range(n):
        tx, ty = (slopes if slopes is not None else (rng.integers(-40, 41) / 128.0, rng.integers(-40, 41) / 128.0))
        if tx == 0 and ty == 0:
            tx = 0.25
        d = (0.0, 2.0, -1.5)[k % 3]
        rows.append([P[0] + tx * d, P[1] + ty * d, P[2] + d, tx, ty, var, 0, 0])
    return np.array(rows)


def test_adversarial_events():
    rng = np.random.default_rng(21)
    evs = []
    evs.append(np.zeros((0, 8)))                                            # empty
    evs.append(np.array([[0.01, 0.02, 3.0, 0.2, 0.1, 1e-3, 0, 0]]))         # one track
    par = np.zeros((40, 8))                                                 # parallel to the beam
    par[:, 2] = rng.uniform(-10, 10, 40)
    par[:, 5] = 1e-3
    evs.append(par)
    evs.append(_exact_event((0.0, 0.0, 12.0), 30, rng, slopes=(0.25, 0.0)))  # identical slopes: singular fit
    wide = np.zeros((60, 8))                                                # wide tracks at the ends
    wide[:30, 2] = rng.uniform(-600, -590, 30)
    wide[:30, 3] = rng.choice([0.004, -0.005], 30)
    wide[:30, 5] = 1e-3
    wide[30:, 2] = rng.uniform(396, 399.99, 30)
    wide[30:, 3] = rng.choice([0.03, -0.025], 30)
    wide[30:, 5] = 1e-3
    evs.append(wide)
    bad = _exact_event((0.0, 0.0, -20.0), 25, rng)                          # NaN, Inf, zero/negative variance
    bad[0, 0] = np.nan
    bad[1, 4] = np.inf
    bad[2, 5] = 0.0
    bad[3, 5] = -1e-3
    bad[4, 7] = np.nan
    evs.append(bad)
    evs.append(_exact_event((0.0, 0.0, 100.0), 25, rng) + 0.0)              # noise-free vertex
    two = np.concatenate([_exact_event((0.0, 0.0, 30.0), 20, rng), _exact_event((0.0, 0.0, 31.0), 20, rng)])
    evs.append(two)                                                         # two vertices 1 mm apart
    b = synth.from_tracks(evs)
    g, o, _ = check(b, name="adversarial")
    assert g.status[3] == pv.PV_EV_FIT_FAILED and g.n_vertices[3] == 0   # the identical-slopes event


@pytest.mark.parametrize("sched", [(2, 512, 4), (8, 1536, 4), (1, 256, 2)], ids=["w2c512m4", "w8c1536m4", "w1c256m2"])
def test_single_event_batches(sched):
    """Batches of one event (no ordering launch): a mu = 5 event, a mu = 40 one
    and one of ~2,500 tracks, which only the large-event launch holds."""
    s = dict(waves_per_team=sched[0], track_capacity=sched[1], persistent=sched[2], teams_per_cu=0)
    for name, b in (("mu5", synth.generate("pp_mu5_10kev", n_events=1, first_event=6, keep_truth=False)),
                    ("mu40", synth.generate("pp_mu40_20kev", n_events=1, first_event=3, keep_truth=False)),
                    ("mu100", synth.generate("pp_mu40_20kev", n_events=1, mu=100.0, keep_truth=False))):
        g, o, _ = check(b, schedule=s, name=f"one {name} event ({b.n_tracks} tracks), schedule {sched}")
        assert g.n_vertices[0] > 0


@pytest.mark.parametrize("persistent", [2, 4], ids=["batch_order", "sorted"])
def test_empty_and_tiny_events_over_several_ordering_slices(persistent):
    """1,500 empty events (two ordering slices, no tracks at all), then 1,100
    events alternating empty, one to three tracks and whole mu = 5 events:
    every event must report no vertex or the oracle's, in either order."""
    rng = np.random.default_rng(33)
    sched = dict(waves_per_team=2, track_capacity=512, persistent=persistent, teams_per_cu=0)
    b = synth.from_tracks([np.zeros((0, 8)) for _ in range(1500)])
    g, o, _ = check(b, schedule=sched, name=f"1500 empty events, mode {persistent}")
    assert not np.any(g.n_vertices) and not np.any(g.status)
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
    b = synth.from_tracks(evs)
    g, o, _ = check(b, schedule=sched, name=f"1100 mixed empty/tiny/mu5 events, mode {persistent}")
    assert np.all(g.n_vertices[0::3] == 0)


@pytest.mark.parametrize("mode", [0, 1], ids=["partition", "multivertex"])
def test_failed_fits_are_flagged(mode):
    """Candidates whose fit fails (tracks along one line: a singular normal
    matrix; tracks all 5 mm from the beam at one z: no Tukey weight at the
    seed) are dropped and flag their event, as in the oracle; the good vertex
    beside them is written."""
    rng = np.random.default_rng(33)
    evs = []
    for z0 in (-300.0, -40.0, 60.0, 250.0):
        good = _exact_event((0.0, 0.0, z0), 15, rng)
        line = np.array([[0.25 * d, -0.125 * d, z0 + 80.0 + d, 0.25, -0.125, 2.0 ** -11, 0, 0]
                         for d in (0.0, 2.0, -1.5, 1.0) * 3])
        off = np.array([[px + tx * d, py + ty * d, z0 - 70.0 + d, tx, ty, 2.0 ** -11, 0, 0]
                        for k, d in enumerate((0.0, 2.0, -1.5) * 4)
                        for (px, py, tx, ty) in [((5.0, 0.0, 0.0, 0.25), (0.0, 5.0, -0.125, 0.0),
                                                  (-5.0, 0.0, 0.0, -0.375), (0.0, -5.0, 0.25, 0.0))[k % 4]]])
        evs += [good, np.concatenate([good, line]), np.concatenate([off, good]), np.concatenate([line, good, off])]
    b = synth.from_tracks(evs)
    g, o, _ = check(b, {"assoc_mode": mode}, name=f"failed fits, mode {mode}")
    flagged = (g.status & pv.PV_EV_FIT_FAILED) != 0
    assert not np.any(flagged[0::4]) and np.all(flagged[1::4]) and np.all(flagged[2::4]) and np.all(flagged[3::4])
    assert np.all(g.n_vertices == 1)


def _ill_conditioned_event(zs, n, rng, slope_sd=3e-4, sxy=1e-4):
    """Vertices on the beamline whose tracks have slopes of order slope_sd:
    z is weakly constrained, so the normal matrix A of Eq. 11 has a 1-norm
    condition number of about 1 / <t^2>, 4e6-9e6 here; sxy = 1e-4 mm keeps
    sigma_poca = sxy / |t| below the 1.5 mm histogram cut."""
    rows = []
    for z in zs:
        t = rng.normal(0.0, slope_sd, (n, 2))
        dz = rng.uniform(-2.0, 2.0, n)
        x = t[:, 0] * dz + rng.normal(0.0, sxy, n)
        y = t[:, 1] * dz + rng.normal(0.0, sxy, n)
        rows.append(np.stack([x, y, z + dz, t[:, 0], t[:, 1], np.full(n, sxy * sxy), np.zeros(n), np.zeros(n)], 1))
    return np.concatenate(rows)


def _kappa1(cov):
    """1-norm condition number of A = C^-1 from a covariance record."""
    c = np.asarray(cov, dtype=np.float64)
    C = np.array([[c[0], c[1], c[3]], [c[1], c[2], c[4]], [c[3], c[4], c[5]]])
    A = np.linalg.inv(C)
    return np.abs(A).sum(0).max() * np.abs(C).sum(0).max()


@pytest.mark.parametrize("mode", [0, 1], ids=["partition", "multivertex"])
def test_fp64_covariance_inversion_on_ill_conditioned_clusters(mode):
    """Eq. 14 in binary64 on the GPU where the condition number of A exceeds
    cond_fp64 = 1e6: every vertex of the constructed events (kappa_1 4e6-9e6 by
    the oracle's covariance) carries PV_VX_FP64_INVERSION, the vertices of
    ordinary mu = 5 events (kappa_1 well below 1e6) do not, and all match the
    oracle to the usual bars (covariance within COV_RTOL)."""
    rng = np.random.default_rng(90)
    ill = synth.from_tracks([_ill_conditioned_event((-100.0, 0.0, 150.0), 25, rng) for _ in range(20)])
    b = synth.concat([ill, synth.generate("pp_mu5_100ev", n_events=30)])
    prm = {"assoc_mode": mode}
    g, o = run_both(b, prm, name=f"fp64 inversion, assoc_mode {mode}")
    rep = parity.compare(b, g, o, debug=True, mv=bool(mode))
    say(f"fp64 inversion: {rep.summary()}")
    assert rep.ok(), "\n".join(rep.problems)
    assert rep.ties <= 2
    n_ill = n_plain = 0
    for e in range(b.n_events):
        for k in range(int(o.n_vertices[e])):
            kap = _kappa1(o.vertices[e, k]["cov"])
            flagged = bool(g.vertices[e, k]["flags"] & pv.PV_VX_FP64_INVERSION)
            if kap > 1.2e6:
                assert flagged, (e, k, kap)
                n_ill += 1
            elif kap < 0.8e6:
                assert not flagged, (e, k, kap)
                n_plain += 1
    say(f"fp64 inversion: {n_ill} vertices inverted in binary64, {n_plain} in binary32")
    assert n_ill == 60 and n_plain > 100


def test_events_larger_than_a_small_team_and_too_many_tracks():
    big = synth.generate("pp_mu40_20kev", n_events=6, mu=150.0)             # ~3900 tracks each
    sizes = np.diff(big.offsets)
    say(f"large events sizes {sizes.tolist()}")
    b = synth.concat([synth.generate("pp_mu5_100ev", n_events=5), big])
    check(b, name="large events")
    lim = int(np.sort(sizes)[2])
    check(b, {"max_tracks_per_event": lim}, name=f"too many tracks (limit {lim})")


def test_event_at_the_track_limit():
    """An event of exactly 4096 tracks (the most an event may have, held by
    one large-event team) matches the oracle; one of 4097 is flagged
    PV_EV_TOO_MANY_TRACKS with its tracks unassigned, on both sides."""
    big = synth.generate("pp_mu40_20kev", n_events=3, mu=150.0)
    rows = np.stack([np.asarray(getattr(big, f), dtype=np.float64) for f in synth.TRACK_FIELDS], 1)
    assert rows.shape[0] >= 4097
    b = synth.concat([synth.generate("pp_mu5_100ev", n_events=3),
                      synth.from_tracks([rows[:4096], rows[:4097]])])
    g, o, _ = check(b, name="4096 and 4097 tracks")
    assert (o.status[-2] & oracle.EV_TOO_MANY_TRACKS) == 0 and o.n_vertices[-2] > 50
    assert (o.status[-1] & oracle.EV_TOO_MANY_TRACKS) != 0 and g.n_vertices[-1] == 0
    assert np.all(g.track_vertex[-4097:] == -1)


def test_largest_batch_sampled_against_the_oracle():
    """300,000 events at mu = 5 (39 M tracks; beyond the allocation-free
    entry point's limit) in one call: the ordering launch runs over many
    chunks of its counting sort and the main grid over 300,000 workgroups.
    600 sampled events, each recomputed by the oracle alone, match."""
    b = synth.generate_parallel("pp_mu5_10kev", n_events=300000)
    say(f"largest batch: {b.n_events} events, {b.n_tracks} tracks")
    g = pv.run(b)
    rng = np.random.default_rng(50)
    sample = np.sort(rng.choice(b.n_events, 600, replace=False))
    sub = b.select(sample)
    tracks = np.concatenate([np.arange(b.offsets[e], b.offsets[e + 1]) for e in sample])
    gs = pv.HostResult(n_vertices=g.n_vertices[sample], status=g.status[sample], vertices=g.vertices[sample],
                       track_vertex=g.track_vertex[tracks], track_weight=g.track_weight[tracks])
    o = oracle.find(sub, parity.oracle_params(pv.pv_params_default()))
    rep = parity.compare(sub, gs, o, debug=False)
    say(f"largest batch sample: {rep.summary()}")
    assert rep.ok(), "\n".join(rep.problems)
    assert rep.ties <= max(2, 0.01 * rep.n_vertices)


def _spread_event(zs, per_vertex, rng):
    return np.concatenate([_exact_event((0.0, 0.0, float(z)), per_vertex, rng) for z in zs])


@pytest.mark.skip(reason="hung on the GPU under a single-wavefront kernel that has since been taken out of the "
                         "library; the hang's cause was not found (a CPU emulation of the kernels on these inputs "
                         "terminates and matches the oracle), so these inputs stay off the GPU")
@pytest.mark.parametrize("sched", WAVE, ids=lambda s: f"c{s['track_capacity']}m{s['persistent']}")
def test_single_wavefront_deferrals(sched):
    """Events the single-wavefront kernel hands to the large-team launch:
    more touched 64-bin words than its 16 pages, more clusters than its 32
    vertex slots, more tracks than its capacity; and the largest events it
    keeps (16 pages, 32 clusters).  Results must match the oracle and, for the
    integer outputs, a multi-wavefront schedule."""
    rng = np.random.default_rng(31)
    evs = [
        _spread_event(np.linspace(-500, 300, 20), 6, rng),     # 20 words, 20 clusters: pages
        _spread_event(np.linspace(-560, 380, 40), 5, rng),     # 40 words, 40 clusters: both
        _spread_event(-592.0 + 16.0 * np.arange(16), 5, rng),  # 16 words exactly, 16 clusters: kept
        _spread_event(-590.0 + 6.0 * np.arange(32), 5, rng),   # 32 clusters in few words: kept
        _spread_event(-590.0 + 6.0 * np.arange(34), 5, rng),   # 34 clusters: vertex slots
        _exact_event((0.0, 0.0, 5.0), 700, rng),               # 700 tracks: capacity
        _exact_event((0.0, 0.0, -5.0), 300, rng),              # 300 tracks: capacity 256 only
    ]
    b = synth.concat([synth.generate("pp_mu5_100ev", n_events=6), synth.from_tracks(evs)])
    g, _, _ = check(b, schedule=sched, name=f"wave deferrals {sched}")
    t = pv.run(b, schedule=TEAM, debug=True)
    assert np.array_equal(g.track_vertex, t.track_vertex) and np.array_equal(g.n_vertices, t.n_vertices)
    assert np.array_equal(g.hist, t.hist) and np.array_equal(g.status, t.status)
    # fewer vertex slots than the kernel holds: overflow flagged, not deferred
    check(b, {"max_vertices_per_event": 24}, schedule=sched, name="wave, 24 vertex slots")


PERSISTENT_HUNG = ("a persistent small-team launch handing events to the large-team launch part-way did not finish "
                   "on the GPU (cause not found; a CPU emulation of the kernels on these inputs terminates and "
                   "matches the oracle); persistent small-team modes are rejected by the library")


@pytest.mark.parametrize("sched", [dict(waves_per_team=2, track_capacity=512, persistent=4, teams_per_cu=0),
                                   pytest.param(dict(waves_per_team=2, track_capacity=512, persistent=1,
                                                     teams_per_cu=0), marks=pytest.mark.skip(reason=PERSISTENT_HUNG)),
                                   dict(waves_per_team=1, track_capacity=256, persistent=2, teams_per_cu=0)],
                         ids=lambda s: f"w{s['waves_per_team']}c{s['track_capacity']}m{s['persistent']}")
def test_small_team_deferrals_within_the_track_limit(sched):
    """Events a small team hands to the large-team launch although they are
    within max_tracks_per_event: 32 touched 64-bin words (more than its 20
    pages) and 72 clusters (more than its 64 vertex slots)."""
    rng = np.random.default_rng(41)
    evs = [_spread_event(np.linspace(-450, 380, 30), 5, rng),
           _spread_event(-598.0 + 4.0 * np.arange(72), 4, rng)]
    b = synth.concat([synth.generate("pp_mu5_100ev", n_events=8), synth.from_tracks(evs)])
    g, o, _ = check(b, {"max_tracks_per_event": 512}, schedule=sched, name=f"small-team deferrals {sched}")
    assert list(o.n_vertices[-2:]) == [30, 72] and list(g.n_vertices[-2:]) == [30, 72]


def test_vertex_overflow_and_region_parameters():
    b = synth.generate("pp_mu5_gas_50kev", n_events=60)
    check(b, {"max_vertices_per_event": 3}, name="overflow, 3 vertex slots")
    check(b, {"z_min": -550.0, "z_max": 300.0}, name="paper histogram range")


def test_invalid_offsets():
    b = synth.generate("pp_mu5_100ev", n_events=4)
    n = b.n_tracks
    o1 = b.offsets.copy()
    k = int(o1[2])
    offs = np.array([0, int(o1[1]), -1, k, n], dtype=np.int32)               # events 1, 2 invalid
    bb = synth.TrackBatch(offsets=offs, **{f: getattr(b, f) for f in synth.TRACK_FIELDS})
    check(bb, name="invalid offsets")
    offs = np.array([0, int(o1[1]), n + 5, n], dtype=np.int32)
    bb = synth.TrackBatch(offsets=offs, **{f: getattr(b, f) for f in synth.TRACK_FIELDS})
    check(bb, name="offsets beyond the track count")


@pytest.mark.parametrize("sched", SCHEDULES, ids=lambda s: f"w{s['waves_per_team']}c{s['track_capacity']}m{s['persistent']}")
def test_schedules_agree(sched):
    b = synth.generate("pp_mu5_100ev", n_events=60)
    g, o, rep = check(b, schedule=sched, debug=True, name=f"schedule {sched}")
    g2 = pv.run(b, schedule=sched, debug=True)
    # same schedule twice: bit-identical, floats included
    assert np.array_equal(g.track_weight.view(np.uint32), g2.track_weight.view(np.uint32))
    assert np.array_equal(g.n_vertices, g2.n_vertices)
    for e in range(b.n_events):   # slots past an event's vertex count are not written
        n = int(g.n_vertices[e])
        assert np.array_equal(g.vertices[e, :n].view(np.uint8), g2.vertices[e, :n].view(np.uint8)), e
    # integer outputs identical to the default schedule
    g0 = pv.run(b, debug=True)
    assert np.array_equal(g.track_vertex, g0.track_vertex) and np.array_equal(g.n_vertices, g0.n_vertices)
    assert np.array_equal(g.hist, g0.hist)


def test_track_order_and_batch_composition_invariance():
    b = synth.generate("pp_mu5_100ev", n_events=40)
    g = pv.run(b, debug=True)
    rng = np.random.default_rng(22)
    perm = np.concatenate([b.offsets[e] + rng.permutation(b.offsets[e + 1] - b.offsets[e])
                           for e in range(b.n_events)])
    bs = synth.TrackBatch(offsets=b.offsets.copy(), **{f: getattr(b, f)[perm] for f in synth.TRACK_FIELDS})
    say("shuffled tracks")
    gs = pv.run(bs, debug=True)
    assert np.array_equal(g.hist, gs.hist) and np.array_equal(g.n_vertices, gs.n_vertices)
    assert np.array_equal(g.track_vertex[perm], gs.track_vertex)
    assert np.max(np.abs(g.track_weight[perm] - gs.track_weight)) < parity.W_TOL
    # an event alone equals the same event inside the batch, bit for bit
    for e in (0, 17, 39):
        say(f"event {e} alone")
        ga = pv.run(b.event(e), debug=True)
        n = int(g.n_vertices[e])
        assert int(ga.n_vertices[0]) == n
        assert np.array_equal(ga.vertices[0, :n].view(np.uint8), g.vertices[e, :n].view(np.uint8))
        a0, a1 = b.offsets[e], b.offsets[e + 1]
        assert np.array_equal(ga.track_weight.view(np.uint32), g.track_weight[a0:a1].view(np.uint32))


def test_config2_full_size_bench_launch():
    """10,000 events at mu = 5 in the benchmark's launch configuration (default
    schedule, no debug outputs), every event compared with the oracle."""
    b = synth.generate("pp_mu5_10kev", keep_truth=False)
    check(b, debug=False, name="pp mu=5 10k events")


def test_config3_beam_gas_sample():
    b = synth.generate("pp_mu5_gas_50kev", n_events=5000, keep_truth=False)
    check(b, debug=True, name="pp + beam-gas 5k events")


def test_config4_high_pileup_sample():
    b = synth.generate("pp_mu40_20kev", n_events=800, keep_truth=False)
    check(b, debug=True, name="mu=40 800 events")


def _check_full_size_autotuned(workload, name):
    """Every event of a workload compared with the oracle, run (without debug
    outputs) under the schedule pv_autotune picks for that very batch, as
    the benchmark times it."""
    b = synth.generate(workload, keep_truth=False)
    p = pv.pv_params_default()
    db = pv.to_device(b)
    out = pv.alloc_outputs(db, p.max_vertices_per_event)
    before = pv.pv_get_schedule()
    best, us = pv.pv_autotune(db, out, p, reps=3)
    pv.pv_set_schedule(before.waves_per_team, before.track_capacity, before.persistent, before.teams_per_cu)
    say(f"{name}: pv_autotune picks {best} ({us:.1f} us per launch)")
    del db, out
    return check(b, schedule=best, debug=False, name=f"{name} under {best}")


def test_config3_beam_gas_full_size_autotuned():
    """50,000 events at mu = 5 with beam-gas vertices."""
    _check_full_size_autotuned("pp_mu5_gas_50kev", "pp + beam-gas 50k events")


def test_config4_high_pileup_full_size_autotuned():
    """20,000 events at mu = 40 (up to ~1,900 tracks per event)."""
    _check_full_size_autotuned("pp_mu40_20kev", "mu=40 20k events")


@pytest.mark.parametrize("waves", [1, 2])
def test_fit_lane_map_one_dominant_vertex_among_many_small(waves):
    """More than 8 vertices share a team's lanes in proportion to their
    tracks: one 600-track vertex beside 40 vertices of 4 tracks.  At one lane
    per small vertex the minimums overrun a one-wavefront team's 64 lanes, so
    the large vertex's block is halved until they fit; two wavefronts hold
    them without halving.  Capacity 1024, so the team keeps the event."""
    rng = np.random.default_rng(47)
    ev = np.concatenate([_exact_event((0.0, 0.0, 150.0), 600, rng)] +
                        [_exact_event((0.0, 0.0, -120.0 + 6.0 * k), 4, rng) for k in range(40)])
    b = synth.concat([synth.from_tracks([ev, ev[::-1].copy()]), synth.generate("pp_mu5_100ev", n_events=6)])
    sched = dict(waves_per_team=waves, track_capacity=1024, persistent=4, teams_per_cu=0)
    g, o, _ = check(b, schedule=sched, name=f"dominant vertex, W={waves}")
    assert int(o.n_vertices[0]) == 41 and int(g.n_vertices[0]) == 41


@pytest.mark.parametrize("cap", [1024, 2048])
def test_config4_high_pileup_one_wavefront_teams(cap):
    """High pile-up on one-wavefront teams: the proportional lane map with a
    64-lane budget."""
    b = synth.generate("pp_mu40_20kev", n_events=300, keep_truth=False)
    check(b, schedule=dict(waves_per_team=1, track_capacity=cap, persistent=4, teams_per_cu=0), debug=True,
          name=f"mu=40 300 events, one wavefront, capacity {cap}")


@pytest.mark.parametrize("cap", [1536, 2048])
def test_config4_high_pileup_large_teams(cap):
    """High pile-up under the schedules that suit it: four-wavefront teams
    holding 1536 or 2048 tracks; with 1536 the few larger events (about 1 %)
    go to the large-event launch."""
    b = synth.generate("pp_mu40_20kev", n_events=800, keep_truth=False)
    check(b, schedule=dict(waves_per_team=4, track_capacity=cap, persistent=4, teams_per_cu=0), debug=True,
          name=f"mu=40 800 events, capacity {cap}")


@pytest.mark.parametrize("n_events", [1025, 40007])
def test_sorted_launch_over_several_ordering_chunks(n_events):
    """The ordering launch sorts slices of at most 1,024 events, one workgroup
    each, and interleaves their ranks: 1,025 events are two slices (513 and
    512), 40,007 are forty (seven of 1,001, the rest of 1,000), so the order
    must still be a permutation of the batch; every event is compared."""
    b = synth.generate("pp_mu5_gas_50kev", n_events=n_events, keep_truth=False)
    check(b, schedule=dict(waves_per_team=2, track_capacity=512, persistent=4, teams_per_cu=0), debug=False,
          name=f"pp + beam-gas {n_events} events, sorted")
