"""GPU parity of the x86 splitting of proto-clusters (Sec. 3.3: the smallest
significant minimum between the two largest maxima, recursively;
`peak_mode = PV_PEAK_RECURSIVE`) against the oracle's same mode, with the
partition association and with the multi-vertex variant."""
import sys

import numpy as np
import pytest

import oracle
import parity
from paper_2412_14966_amd import pvfind as pv, synth
from test_gpu_parity import _exact_event

pytestmark = pytest.mark.gpu

REC = {"peak_mode": 1}


def say(msg):
    print(f"[gpu-rec] {msg}", flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module", autouse=True)
def _gpu():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    pv.lib()
    yield


def triplets(n, seed=48):
    """Events of three exact vertices 0.5-2 mm apart, the middle one small:
    with a cluster-integral threshold of 6 tracks the two splittings give
    different clusters on a few percent of them."""
    rng = np.random.default_rng(seed)
    evs = []
    for _ in range(n):
        z0 = rng.uniform(-200, 200)
        d1, d2 = rng.uniform(0.5, 2.0, 2)
        k = rng.integers([8, 3, 8], [25, 9, 25])
        evs.append(np.concatenate([_exact_event((0, 0, z0), k[0], rng), _exact_event((0, 0, z0 + d1), k[1], rng),
                                   _exact_event((0, 0, z0 + d1 + d2), k[2], rng)]))
    return synth.from_tracks(evs)


def check(batch, params, schedule=None, debug=True, name=""):
    p = pv.make_params(params)
    mv = bool(params.get("assoc_mode", 0))
    say(f"{name}: {batch.n_events} events, {batch.n_tracks} tracks, params={params}, schedule={schedule}")
    g = pv.run(batch, params, schedule=schedule, debug=debug)
    o = oracle.find(batch, parity.oracle_params(p), debug=debug)
    rep = parity.compare(batch, g, o, debug=debug, mv=mv)
    say(f"{name}: {rep.summary()}")
    assert rep.ok(), "\n".join(rep.problems)
    assert rep.ties <= max(3, 0.01 * rep.n_vertices)
    return g, o


@pytest.mark.parametrize("sched", [None, dict(waves_per_team=1, track_capacity=256, persistent=2, teams_per_cu=0)],
                         ids=["default", "w1c256m2"])
def test_recursive_split_where_the_variants_differ(sched):
    b = triplets(300)
    prm = {"min_int_pp": 6 * 65536}
    _, o_zo = check(b, prm, sched, name="z-ordered")
    _, o_rc = check(b, dict(prm, **REC), sched, name="recursive")
    differ = sum(int(o_zo.n_clusters[e]) != int(o_rc.n_clusters[e]) or
                 not np.array_equal(o_zo.clusters[e, :o_zo.n_clusters[e]]["hi"],
                                    o_rc.clusters[e, :o_rc.n_clusters[e]]["hi"]) for e in range(b.n_events))
    say(f"events whose clusters differ between the splittings: {differ}")
    assert differ >= 3


def test_recursive_split_on_the_workloads():
    check(synth.generate("pp_mu5_100ev"), REC, name="recursive mu=5")
    check(synth.generate("pp_mu40_20kev", n_events=300, keep_truth=False), REC, name="recursive mu=40")
    check(synth.generate("pp_mu5_gas_50kev", n_events=2000, keep_truth=False), dict(REC, assoc_mode=1),
          name="recursive + multi-vertex, beam-gas")
