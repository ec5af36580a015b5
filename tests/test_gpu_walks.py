"""Walk bookkeeping on the GPU: the node-visit bound on small meshes walked
by many segments, the deep pass that finishes walks whose stack outgrows
its LDS part, the all-hits lists collected during the walk (library or
caller pool, overflow detection, batches and captured graphs), and the
stream-ordered build whose index check is reported by rsi_query_stats.
Every case is compared with the FP64 oracle or with a path already held to
it, bit for bit (the paper's Section 3.2 traversal and candidate buffer,
Section 3.3 kernel)."""
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


def _soup(n_t, seed):
    """n_t random triangles in the unit cube (their own three vertices each)."""
    rng = np.random.default_rng(seed)
    V = rng.uniform(0.0, 1.0, size=(3 * n_t, 3)).astype(np.float32)
    T = np.arange(3 * n_t, dtype=np.int32).reshape(n_t, 3)
    return V, T


def _lists(sp, base=0):
    """{segment: (ids, ts)} of a spill read-back (segment ids offset by -base)."""
    if sp is None:
        return {}
    seg, off, cnt = (sp[k].cpu().numpy() for k in ("seg", "offset", "count"))
    ids, ts = sp["ids"].cpu().numpy(), sp["ts"].cpu().numpy()
    return {int(s) - base: (ids[o:o + c].tolist(), ts[o:o + c].tolist()) for s, o, c in zip(seg, off, cnt)}


@pytest.mark.parametrize("n_t", [3, 4, 5, 8, 16, 40])
def test_small_meshes_many_segments(n_t):
    """A tiny tree walked by 2M segments: waves run many rounds per segment
    set, and no walk may be cut short; every non-degenerate segment must
    match the oracle in the boolean, first-hit and all-hits modes."""
    V, T = _soup(n_t, 100 + n_t)
    rng = np.random.default_rng(200 + n_t)
    n = 2_000_000
    S, E = wl.segments_in_box(rng, [-0.2] * 3, [1.2] * 3, n)
    print(f"n_t={n_t} n_r={n}", flush=True)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    out = mesh.query(_t(S), _t(E), "bool|first|all", capacity=4)
    st = mesh.stats()
    assert st["walk_cut"] == 0 and st["stack_dropped"] == 0
    ref = parity.oracle_reference(V, T, S, E, cap=4)
    spill = out.get("spill")
    if spill is not None:
        segs = spill["seg"].cpu().numpy()
        full = parity.oracle.query(V, T, S[np.sort(segs)], E[np.sort(segs)], cap=64)
        ref["full_lists"] = {int(s): [(full["list_t"][k, j], int(full["list_tri"][k, j]))
                                      for j in range(full["count"][k])] for k, s in enumerate(np.sort(segs))}
    rep = parity.compare(ref, out, {"bool", "first", "all"}, cap=4, spill=spill)
    print(rep)
    parity.assert_parity(rep)
    assert rep["hits"] > n // 20
    mesh.close()


def test_deep_pass_matches_main_pass():
    """A two-entry LDS stack sends most walks of the closed sphere to the
    deep pass (stack continued in device memory); every answer must equal
    the default stack's, in every mode."""
    V, T = wl.noisy_sphere(40, 8, 0.3)
    rng = np.random.default_rng(31)
    S, E = wl.segments_in_box(rng, V.min(0), V.max(0), 300_000, scale=1.5)
    Vt, Tt, St, Et = _t(V), _t(T, torch.int32), _t(S), _t(E)
    for branching in (4, 2):
        base = rsi.Mesh(Vt, Tt, branching=branching)
        small = rsi.Mesh(Vt, Tt, branching=branching, stack_depth=2)
        for mode in ("bool", "first", "count", "all|first"):
            a = base.query(St, Et, mode, capacity=2)
            deep0 = base.stats()["deep_segments"]
            b = small.query(St, Et, mode, capacity=2)
            st = small.stats()
            print(branching, mode, "deep segments:", deep0, st["deep_segments"], flush=True)
            assert st["deep_segments"] > 10_000, (branching, mode)
            for k in a:
                if k == "spill":
                    assert _lists(a[k]) == _lists(b[k]), (branching, mode)
                else:
                    assert torch.equal(a[k], b[k]), (branching, mode, k)
        base.close()
        small.close()


def test_caller_pool_and_overflow_detection():
    """All hits into a caller pool: the same lists as the library pool,
    spill_off pointing at them; a pool too small gives RSI_E_OVERFLOW with
    exact counts and every list that fitted intact."""
    V, T = wl.noisy_sphere(24, 99, 0.3)
    rng = np.random.default_rng(5)
    S, E = wl.segments_in_box(rng, V.min(0), V.max(0), 50_000, scale=1.5)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    St, Et = _t(S), _t(E)
    lib = mesh.query(St, Et, "all", capacity=1)
    want = _lists(lib["spill"])
    n_over = len(want)
    total = sum(len(v[0]) for v in want.values())
    assert n_over > 1000
    for cap_pool, expect_full in ((total + 10, False), (total // 3, True)):
        out = mesh.alloc_outputs(S.shape[0], "all", capacity=1)
        out["spill_off"] = torch.empty(S.shape[0], dtype=torch.int64, device=DEV)
        out["spill_ids"] = torch.full((cap_pool,), -7, dtype=torch.int32, device=DEV)
        out["spill_ts"] = torch.zeros(cap_pool, dtype=torch.float32, device=DEV)
        mesh.query_into(St, Et, "all", out, capacity=1)
        st = mesh.stats(check=False)
        assert torch.equal(out["count"], lib["count"])
        assert st["overflow_crossings"] == total
        soff = out["spill_off"].cpu().numpy()
        cnt = out["count"].cpu().numpy()
        ids, ts = out["spill_ids"].cpu().numpy(), out["spill_ts"].cpu().numpy()
        got = {int(i): (ids[soff[i]:soff[i] + cnt[i]].tolist(), ts[soff[i]:soff[i] + cnt[i]].tolist())
               for i in np.nonzero(soff >= 0)[0]}
        assert np.all(soff[cnt <= 1] == -1)
        for i, v in got.items():
            assert v == want[i], i
        if expect_full:
            assert st["status"] == rsi.RSI_E_OVERFLOW and st["overflow_full"] == 1
            assert 0 < len(got) < n_over
            # slots of the segments without room are marked empty
            lost = (cnt > 1) & (soff < 0)
            assert np.all(out["ids"].cpu().numpy()[lost, 0] == -1)
        else:
            assert st["status"] == rsi.RSI_OK and len(got) == n_over
            assert torch.equal(out["ids"], lib["ids"]) and torch.equal(out["ts"], lib["ts"])
    mesh.close()


def _batch_workloads():
    ws = wl.config5(n_meshes=8, tri_lo=500, tri_hi=20_000, seg_lo=2_000, seg_hi=30_000, seed=77)
    meshes = [(_t(w.V), _t(w.T, torch.int32)) for w in ws]
    segs = [(_t(w.S), _t(w.E)) for w in ws]
    return ws, meshes, segs


def test_batch_all_hits_equals_sequential():
    ws, meshes, segs = _batch_workloads()
    b = rsi.Batch(meshes)
    outs = b.query(segs, "all|first", capacity=2)
    blists = _lists(outs[0].get("spill"))
    base = 0
    for k, ((V, T), (S, E)) in enumerate(zip(meshes, segs)):
        m = rsi.Mesh(V, T)
        ref = m.query(S, E, "all|first", capacity=2)
        for key in ("count", "ids", "ts", "tri", "t", "uv", "point"):
            assert torch.equal(outs[k][key], ref[key]), (ws[k].name, key)
        n = S.shape[0]
        mine = {s - base: v for s, v in blists.items() if base <= s < base + n}
        assert mine == _lists(ref.get("spill")), ws[k].name
        base += n
        m.close()
    b.close()


def test_graph_all_hits_replays_match_eager():
    ws, meshes, segs = _batch_workloads()
    b = rsi.Batch(meshes)
    eager = b.query(segs, "all|bool", capacity=3)
    outs = b.alloc_outputs(segs, "all|bool", capacity=3)
    b.capture(segs, "all|bool", outs, rebuild=True)
    for rep in range(3):
        for d in outs:
            for v in d.values():
                v.zero_()
        b.replay()
        st = b.stats()
        assert st["status"] == rsi.RSI_OK
        for k in range(len(ws)):
            for key in ("hit", "count", "ids", "ts"):
                assert torch.equal(outs[k][key], eager[k][key]), (rep, ws[k].name, key)
        assert _lists(rsi.read_spill(b.handle)) == _lists(eager[0].get("spill"))
        _ = b.query(segs, "bool")  # eager work between replays
        torch.cuda.synchronize()
    b.close()


def test_captured_rebuild_follows_moved_vertices():
    """A graph captured with its rebuild, replayed after the vertices moved
    (the trees change shape and height): the replay must equal a fresh build
    and query of the moved meshes, and the oracle on samples."""
    ws, meshes, segs = _batch_workloads()
    b = rsi.Batch(meshes)
    outs = b.alloc_outputs(segs, "bool|first")
    b.capture(segs, "bool|first", outs, rebuild=True)
    b.replay()
    torch.cuda.synchronize()
    for step, scale in enumerate((1.7, 0.05)):
        for V, _ in meshes:
            V.mul_(torch.tensor([1.0, 1.0, scale], device=DEV))
        b.replay()
        torch.cuda.synchronize()
        for k, ((V, T), (S, E)) in enumerate(zip(meshes, segs)):
            m = rsi.Mesh(V, T)
            ref = m.query(S, E, "bool|first")
            for key in ref:
                assert torch.equal(outs[k][key], ref[key]), (step, ws[k].name, key)
            m.close()
            idx = wl.subset(S.shape[0], 300, 50 + k)
            Vn = V.cpu().numpy()
            orc = parity.oracle_reference(Vn, ws[k].T, S.cpu().numpy()[idx], E.cpu().numpy()[idx])
            rep = parity.compare(orc, {key: outs[k][key].cpu().numpy()[idx] for key in outs[k]},
                                 {"bool", "first"})
            parity.assert_parity(rep)
    b.close()


def test_build_is_stream_ordered_and_reports_bad_index_later():
    V = _t(np.zeros((3, 3), np.float32))
    bad = _t(np.array([[0, 1, 3]], np.int32), torch.int32)
    m = rsi.Mesh(V, bad, check=False)  # returns without waiting
    S = torch.zeros(4, 3, device=DEV)
    m.query(S, S + 1, "bool")          # the index never reaches past V
    with pytest.raises(rsi.RsiError):
        m.stats()
    m.close()
    good = rsi.Mesh(V, _t(np.array([[0, 1, 2]], np.int32), torch.int32), check=False)
    assert good.stats()["bad_index"] == 0
    good.close()
