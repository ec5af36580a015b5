"""Work counters of the query kernel (its counting variant).

The counting variant runs the same walk with per-lane and per-wave tallies:
its answers must equal the plain kernel's, every segment must be counted
once, and the wave-level tallies must account for every lane slot of every
node step (a lane either visits a node, waits for its pending leaf tests,
or has no node).
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device="cuda", dtype=dtype).contiguous()


@pytest.mark.parametrize("branching", [2, 4])
@pytest.mark.parametrize("mode", ["bool", "first", "all"])
def test_counters_account_for_every_lane(branching, mode):
    w = wl.config1(n_r=60_000)
    V, T, S, E = _t(w.V), _t(w.T, torch.int32), _t(w.S), _t(w.E)
    mesh = rsi.Mesh(V, T, branching=branching)
    ref = mesh.query(S, E, mode, capacity=4)
    mesh.set_counting(True)
    got = mesh.query(S, E, mode, capacity=4)
    torch.cuda.synchronize()
    c = mesh.counters()
    mesh.set_counting(False)
    for k in ref:
        if isinstance(ref[k], torch.Tensor):
            assert torch.equal(ref[k], got[k]), k
    assert c["segments"] == w.n_r
    assert c["node_visits"] + c["lanes_blocked"] + c["lanes_waiting"] == 64 * c["wave_node_steps"]
    if branching == 2:
        assert c["box_tests"] == 2 * c["node_visits"]
    else:
        assert c["node_visits"] <= c["box_tests"] <= 4 * c["node_visits"]
    hits = int((got["hit"] if "hit" in got else (got["count"] > 0) if "count" in got else (got["tri"] >= 0)).sum())
    assert c["tri_tests"] >= hits
    assert 0 < c["wave_refills"] <= c["wave_loops"]
    assert c["wave_leaf_phases"] <= c["wave_leaf_rounds"]
    assert c["wave_leaf_rounds"] <= c["leaf_lanes"] <= 64 * c["wave_leaf_rounds"]
    assert c["leaf_lanes"] <= c["tri_tests"]
    mesh.close()


@pytest.mark.parametrize("n", [1, 2, 7, 8, 9, 63, 65, 257, 1001])
def test_every_segment_claimed_once_at_small_sizes(n):
    """Work items are claimed from eight ranges (one per XCD, some empty at
    these sizes) and stolen across them: every segment must be walked once,
    and the answers must be the oracle's."""
    from tests import parity
    w = wl.config1(n_r=max(n, 16))
    S, E = w.S[:n], w.E[:n]
    V, T = _t(w.V), _t(w.T, torch.int32)
    mesh = rsi.Mesh(V, T)
    mesh.set_counting(True)
    out = mesh.query(_t(S), _t(E), "bool|count")
    torch.cuda.synchronize()
    c = mesh.counters()
    mesh.close()
    assert c["segments"] == n
    ref = parity.oracle_reference(w.V, w.T, S, E)
    ok = ref["degenerate"] == 0
    assert np.array_equal(out["count"].cpu().numpy()[ok], ref["count"][ok])
    assert np.array_equal(out["hit"].cpu().numpy()[ok].astype(bool), ref["count"][ok] > 0)
