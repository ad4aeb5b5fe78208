"""pv_compact_vertices: the written vertex records of a batch, gathered into
one dense array in event order, equal the records pv_find wrote, bit for bit."""
import numpy as np
import pytest

from paper_2412_14966_amd import pvfind as pv
from paper_2412_14966_amd import synth

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("workload,n", [("pp_mu5_10kev", 3000), ("pp_mu40_20kev", 200), ("pp_mu5_100ev", 1)])
def test_compacted_records_equal_the_slots(workload, n):
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    b = synth.generate(workload, n_events=n, keep_truth=False)
    p = pv.pv_params_default()
    db = pv.to_device(b)
    out = pv.alloc_outputs(db, p.max_vertices_per_event)
    pv.pv_find(db, out, p)
    mv = p.max_vertices_per_event
    dense = torch.full((n * mv * 64,), 0xAB, dtype=torch.uint8, device=out.vertices.device)
    first = torch.full((n + 1,), -9, dtype=torch.int32, device=out.vertices.device)
    pv.pv_compact_vertices(out, n, dense, first)
    torch.cuda.synchronize()
    nv = out.n_vertices.cpu().numpy()
    f = first.cpu().numpy()
    assert f[0] == 0 and np.array_equal(np.diff(f), nv) and f[n] == nv.sum()
    slots = out.vertices.cpu().numpy()[:n * mv * 64].reshape(n, mv, 64)
    d = dense.cpu().numpy()
    want = np.concatenate([slots[e, :nv[e]].reshape(-1) for e in range(n)])
    assert np.array_equal(d[:64 * f[n]], want)
    assert np.all(d[64 * f[n]:] == 0xAB)     # nothing written beyond the total
