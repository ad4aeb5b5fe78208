"""Seeded synthetic workloads: shapes, reproducibility and distributions."""
import numpy as np

from paper_2412_14966_amd import synth


def test_event_reproducible_alone_and_in_batch():
    b = synth.generate("pp_mu5_10kev", n_events=20)
    one = synth.generate("pp_mu5_10kev", n_events=1, first_event=13)
    a, z = b.offsets[13], b.offsets[14]
    for f in synth.TRACK_FIELDS:
        assert np.array_equal(getattr(b, f)[a:z], getattr(one, f))
    assert np.array_equal(synth.generate("pp_mu5_10kev", n_events=20).x, b.x)


def test_layout_and_dtypes():
    b = synth.generate("pp_mu5_100ev", n_events=10)
    assert b.offsets.dtype == np.int32 and b.offsets[0] == 0 and np.all(np.diff(b.offsets) >= 0)
    for f in b.fields():
        assert f.dtype == np.float32 and f.shape == (b.n_tracks,)
    assert np.all(b.cov_xx > 0) and np.all(b.cov_xtx == 0) and np.all(b.cov_txtx == 0)


def test_distributions_match_the_workload_description():
    b = synth.generate("pp_mu5_10kev", n_events=2000)
    npv = np.array([len(t) for t in b.truth_pvs])
    assert abs(npv.mean() - 5.0) < 0.15
    nt = np.concatenate(b.truth_ntracks)
    assert abs(nt.mean() - 26.0) < 0.8                 # 1 + NegBin(mean 25, k = 3)
    assert abs(nt.var() - (25 + 25 ** 2 / 3)) < 30
    z = np.concatenate([t[:, 2] for t in b.truth_pvs])
    assert abs(z.std() - 45.0) < 1.5
    x = np.concatenate([t[:, 0] for t in b.truth_pvs])
    assert abs(x.std() - 0.03) < 0.002
    assert abs(b.tx.std() - 0.3) < 0.005
    sxy = np.sqrt(b.cov_xx.astype(np.float64))
    assert sxy.min() >= 0.01 - 1e-7 and sxy.max() <= 0.05 + 1e-7
    mean_tracks = b.n_tracks / b.n_events
    assert 120 < mean_tracks < 140


def test_gas_and_loguniform_workloads():
    g = synth.generate("pp_mu5_gas_50kev", n_events=1500)
    gz = np.concatenate([t[t[:, 3] == 1, 2] for t in g.truth_pvs])
    assert abs(len(gz) / 1500 - 0.5) < 0.06
    assert gz.min() >= -541 and gz.max() <= -341
    gnt = np.concatenate([nt[t[:, 3] == 1] for t, nt in zip(g.truth_pvs, g.truth_ntracks)])
    assert abs(gnt.mean() - 9.0) < 0.8                 # 1 + NegBin(mean 8, k = 2)
    s = synth.generate("served_mulog_200kev", n_events=1500)
    npv = np.array([len(t) for t in s.truth_pvs])
    assert abs(npv.mean() - 39.0 / np.log(40.0)) < 0.6  # E[mu] for mu log-uniform on [1, 40]


def test_select_and_concat_round_trip():
    b = synth.generate("pp_mu5_100ev", n_events=8)
    s = synth.concat([b.select([0, 1, 2]), b.select([3, 4, 5, 6, 7])])
    assert np.array_equal(s.offsets, b.offsets) and np.array_equal(s.ty, b.ty)


def test_parallel_generation_equals_sequential():
    """Events are seeded one by one, so drawing chunks in worker processes
    gives the same batch as drawing them in order."""
    a = synth.generate_parallel("served_mulog_200kev", n_events=700, workers=3, chunk=200)
    b = synth.generate("served_mulog_200kev", n_events=700, keep_truth=False)
    assert np.array_equal(a.offsets, b.offsets)
    for f in synth.TRACK_FIELDS:
        assert np.array_equal(getattr(a, f), getattr(b, f)), f
