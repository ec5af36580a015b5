"""Batched mode: many meshes built by the same launches and queried by one
persistent launch, optionally replayed from a captured HIP graph.  Results
must equal separate per-mesh builds and queries bit for bit, and match the
oracle on samples."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl
from tests import parity

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def _workloads():
    ws = wl.config5(n_meshes=10, tri_lo=500, tri_hi=20_000, seg_lo=2_000, seg_hi=40_000, seed=123)
    # edge cases: an empty mesh and a single triangle
    V1 = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float32)
    rng = np.random.default_rng(2)
    S, E = wl.segments_in_box(rng, [-0.5, -0.5, -1], [1.5, 1.5, 1], 3000)
    ws.append(wl.Workload("single", V1, np.array([[0, 1, 2]], np.int32), S, E))
    ws.append(wl.Workload("empty", np.zeros((0, 3), np.float32), np.zeros((0, 3), np.int32), S[:100], E[:100]))
    return ws


@pytest.fixture(scope="module")
def batch_setup():
    ws = _workloads()
    meshes = [(_t(w.V), _t(w.T, torch.int32)) for w in ws]
    segs = [(_t(w.S), _t(w.E)) for w in ws]
    b = rsi.Batch(meshes)
    return ws, meshes, segs, b


@pytest.mark.parametrize("mode", ["bool", "first", "bool|first"])
def test_batch_equals_sequential(batch_setup, mode):
    ws, meshes, segs, b = batch_setup
    outs = b.query(segs, mode)
    torch.cuda.synchronize()
    for k, ((V, T), (S, E)) in enumerate(zip(meshes, segs)):
        m = rsi.Mesh(V, T)
        ref = m.query(S, E, mode)
        torch.cuda.synchronize()
        for key in ref:
            assert torch.equal(outs[k][key], ref[key]), (ws[k].name, key)
        m.close()


def test_batch_matches_oracle_on_samples(batch_setup):
    ws, meshes, segs, b = batch_setup
    outs = b.query(segs, "bool|first")
    torch.cuda.synchronize()
    for k, w in enumerate(ws):
        idx = wl.subset(w.n_r, 1000, 7 + k)
        ref = parity.oracle_reference(w.V, w.T, w.S[idx], w.E[idx])
        got = {key: outs[k][key].cpu().numpy()[idx] for key in outs[k]}
        rep = parity.compare(ref, got, {"bool", "first"})
        parity.assert_parity(rep)


def test_batch_tree_per_mesh(batch_setup):
    ws, meshes, segs, b = batch_setup
    tree = b.tree()
    order = tree["order"]
    for k, w in enumerate(ws):
        info = b.mesh_info(k)
        lo, n = info["tri_offset"], info["n_t"]
        assert n == w.n_t
        # every sorted leaf of mesh k holds a triangle of mesh k
        assert np.all((order[lo:lo + n] >= lo) & (order[lo:lo + n] < lo + n))
        assert np.array_equal(np.sort(order[lo:lo + n]), np.arange(lo, lo + n))


def test_graph_replay_matches_eager(batch_setup):
    ws, meshes, segs, b = batch_setup
    eager = b.query(segs, "bool|first")
    torch.cuda.synchronize()
    outs = b.alloc_outputs(segs, "bool|first")
    b.capture(segs, "bool|first", outs, rebuild=True)
    for rep in range(4):
        for d in outs:
            for v in d.values():
                v.zero_()
        b.replay()
        torch.cuda.synchronize()
        for k in range(len(ws)):
            for key in eager[k]:
                assert torch.equal(outs[k][key], eager[k][key]), (rep, ws[k].name, key)
        # eager work between replays
        _ = b.query(segs, "bool")
        torch.cuda.synchronize()


def test_batch_rejects_bad_input():
    V = _t(np.zeros((3, 3), np.float32))
    with pytest.raises(rsi.RsiError):
        rsi.Batch([(V, _t(np.array([[0, 1, 3]], np.int32), torch.int32))])


def test_stack_depth_and_tuning_keep_answers(batch_setup, tmp_path):
    """Any LDS stack depth (the rest of the stack in device memory), any
    tuned option set, and the tuner itself leave every answer unchanged."""
    from paper_2209_02878_amd import tune
    ws, meshes, segs, b = batch_setup
    base = b.query(segs, "bool|first")
    for sd in (1, 3, 8):
        b.set_opts(stack_depth=sd)
        out = b.query(segs, "bool|first")
        torch.cuda.synchronize()
        for k in range(len(ws)):
            for key in base[k]:
                assert torch.equal(out[k][key], base[k][key]), (sd, ws[k].name, key)
    best = tune.autotune(b, segs, mode="bool|first", kind="batch", n_t=sum(w.n_t for w in ws),
                         n_r=sum(w.n_r for w in ws), cache_path=str(tmp_path / "c.json"), reps=1)
    applied = b.opts()
    for k, v in best.items():
        if k != "stack_depth" or v:
            assert applied[k] == v, (k, v, applied)
    out = b.query(segs, "bool|first")
    torch.cuda.synchronize()
    for k in range(len(ws)):
        for key in base[k]:
            assert torch.equal(out[k][key], base[k][key]), (ws[k].name, key)
    # a cached shape applies the same options without searching again
    best2 = tune.autotune(b, segs, mode="bool|first", kind="batch", n_t=sum(w.n_t for w in ws),
                          n_r=sum(w.n_r for w in ws), cache_path=str(tmp_path / "c.json"), reps=1)
    assert best2 == best


def test_single_mesh_tuning_and_small_stack():
    w = wl.config1(n_r=30_000)
    m = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    S, E = _t(w.S), _t(w.E)
    base = m.query(S, E, "bool|first|all", capacity=2)
    m.set_opts(stack_depth=2)
    out = m.query(S, E, "bool|first|all", capacity=2)
    for key in ("hit", "tri", "t", "count", "ids", "ts"):
        assert torch.equal(out[key], base[key]), key
    i, ms = m.tune(S, E, "bool|first|all", [{"leaf_size": 2}, {"leaf_size": 1, "block_size": 64}], capacity=2,
                   reps=2)
    assert i in (0, 1) and all(x > 0 for x in ms)
    out = m.query(S, E, "bool|first|all", capacity=2)
    for key in ("hit", "tri", "t", "count", "ids", "ts"):
        assert torch.equal(out[key], base[key]), key
