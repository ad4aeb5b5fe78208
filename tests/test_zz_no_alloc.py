"""The allocation-free entry point pv_find_noalloc against pv_find, called
through the C ABI: two calls in a row on one stream, the second with a
smaller batch (the library's fixed workspace keeps the first call's
contents, whose counters the second call must clear), then a batch whose
large events go through the deferred-event list of that workspace.  For a
fixed schedule the outputs are identical bit for bit."""
import sys

import numpy as np
import pytest

from paper_2412_14966_amd import pvfind as pv
from paper_2412_14966_amd import synth

pytestmark = pytest.mark.gpu


def say(msg):
    print(f"[gpu-noalloc] {msg}", flush=True)
    sys.stdout.flush()


def _run(fn, batch, params):
    import torch
    db = pv.to_device(batch)
    out = pv.alloc_outputs(db, params.max_vertices_per_event)
    out.n_vertices.fill_(-7)
    out.status.fill_(-7)
    out.track_vertex.fill_(-7)
    fn(db, out, params)
    torch.cuda.synchronize()
    return pv.to_host(db, out)


def _same(a, b, batch, max_v):
    assert np.array_equal(a.n_vertices, b.n_vertices)
    assert np.array_equal(a.status, b.status)
    assert np.array_equal(a.track_vertex, b.track_vertex)
    assert np.array_equal(a.track_weight.view(np.uint32), b.track_weight.view(np.uint32))
    for e in range(batch.n_events):
        n = int(a.n_vertices[e])
        assert np.array_equal(a.vertices[e, :n].view(np.uint8), b.vertices[e, :n].view(np.uint8)), e


def test_noalloc_equals_pv_find_on_two_calls_in_a_row():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    params = pv.pv_params_default()
    big = synth.generate("pp_mu5_10kev", n_events=6000, keep_truth=False)
    small = synth.generate("pp_mu5_100ev", n_events=37)
    for name, b in (("6000 events", big), ("37 events", small)):
        say(f"{name}: pv_find_noalloc then pv_find")
        g0 = _run(pv.pv_find_noalloc, b, params)
        g1 = _run(pv.pv_find, b, params)
        _same(g0, g1, b, params.max_vertices_per_event)
        say(f"{name}: {int(g0.n_vertices.sum())} vertices, identical")


def test_noalloc_deferred_events():
    """mu = 40 events larger than the default team go through the deferred
    list held in the fixed workspace."""
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    params = pv.pv_params_default()
    b = synth.generate("pp_mu40_20kev", n_events=300, keep_truth=False)
    say("300 mu=40 events (most deferred to the large-event launch)")
    g0 = _run(pv.pv_find_noalloc, b, params)
    g1 = _run(pv.pv_find, b, params)
    _same(g0, g1, b, params.max_vertices_per_event)
    g2 = _run(pv.pv_find_noalloc, b.select(range(40)), params)
    _same(g2, _run(pv.pv_find, b.select(range(40)), params), b.select(range(40)), params.max_vertices_per_event)
