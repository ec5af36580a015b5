"""The four-way traversal (branching 4) gives exactly the binary walk's answers.

The four-way view lists, for every binary node, the boxes of its
grandchildren (the binary tree of Section 3.1 seen two levels at a time),
quantised outward to 8 bits per plane, so every leaf the exact boxes reach
is reached and the same FP32 triangle test decides; the FP64 re-solve of
every reported crossing is the same too.  The two walks can differ only
where a triangle test sits within rounding of its decision for a triangle
that the looser boxes let through; on these workloads no such case occurs,
so the outputs are compared bit for bit with the binary walk, in every
mode, with a small LDS stack (device-memory tail), with larger leaves,
after a refit, in a batch and in a captured graph; and they must match the
FP64 oracle.
"""
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


def _spill_lists(sp):
    """Per-segment crossing lists of a spill read-back (the order of the
    segments in it depends on timing; each segment's list does not)."""
    seg, off, cnt = (sp[k].cpu().numpy() for k in ("seg", "offset", "count"))
    ids, ts = sp["ids"].cpu().numpy(), sp["ts"].cpu().numpy()
    return {int(s): (ids[o:o + c].tolist(), ts[o:o + c].tolist()) for s, o, c in zip(seg, off, cnt)}


def _equal(a, b, tag):
    for key in a:
        if key == "spill":
            assert _spill_lists(a[key]) == _spill_lists(b[key]), tag
        elif isinstance(a[key], dict):
            _equal(a[key], b[key], tag + "." + key)
        else:
            assert torch.equal(a[key], b[key]), (tag, key)


def _both(mesh, S, E, mode, cap=4):
    mesh.set_opts(branching=2)
    r2 = mesh.query(S, E, mode, capacity=cap)
    mesh.set_opts(branching=4)
    assert mesh.opts()["branching"] == 4
    r4 = mesh.query(S, E, mode, capacity=cap)
    torch.cuda.synchronize()
    return r2, r4


@pytest.mark.parametrize("mode", ["bool", "first", "all|first", "count"])
def test_wide_equals_binary_heightfield(mode):
    w = wl.config2(n_r=200_000)
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    r2, r4 = _both(mesh, _t(w.S), _t(w.E), mode, cap=2)
    _equal(r2, r4, mode)
    mesh.close()


def test_wide_equals_binary_closed_sphere_with_spill_and_small_stack():
    w = wl.config3(n_r=500_000)
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    S, E = _t(w.S), _t(w.E)
    r2, r4 = _both(mesh, S, E, "all|first|bool", cap=2)
    _equal(r2, r4, "sphere")
    assert "spill" in r4
    # four LDS entries: the rest of the stack lives in device memory
    mesh.set_opts(branching=4, stack_depth=4)
    r4s = mesh.query(S, E, "all|first|bool", capacity=2)
    torch.cuda.synchronize()
    _equal(r2, r4s, "sphere-small-stack")
    # the boolean and counting walks (which also read the LDS copy of the top
    # records) with the same four-entry LDS stack
    for mode in ("bool", "count"):
        mesh.set_opts(branching=2, stack_depth=0)
        b2 = mesh.query(S, E, mode)
        mesh.set_opts(branching=4, stack_depth=4)
        b4 = mesh.query(S, E, mode)
        torch.cuda.synchronize()
        _equal(b2, b4, f"sphere-small-stack-{mode}")
    mesh.close()


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6, 9, 16, 17, 21, 22, 64, 85, 86, 300])
def test_wide_small_meshes(n):
    """Triangle soups small enough that the top three four-way levels (the
    records the walk reads from its LDS copy) hold leaves, empty slots and
    missing records: both walks agree bit for bit and match the oracle."""
    rng = np.random.default_rng(1000 + n)
    c = rng.uniform(0.0, 1.0, size=(n, 1, 3))
    V = (c + rng.normal(0.0, 0.15, size=(n, 3, 3))).reshape(-1, 3).astype(np.float32)
    T = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
    S, E = wl.segments_in_box(rng, V.min(0), V.max(0), 3000, scale=1.5)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    r2, r4 = _both(mesh, _t(S), _t(E), "bool|first|all", cap=4)
    _equal(r2, r4, f"n={n}")
    ref = parity.oracle_reference(V, T, S, E, cap=4)
    rep = parity.compare(ref, r4, {"bool", "first", "all"}, cap=4)
    parity.assert_parity(rep)
    # the boolean and counting walks on their own (they take the LDS copy)
    ok = ref["degenerate"] == 0
    for mode, key in (("bool", "hit"), ("count", "count")):
        a2, a4 = _both(mesh, _t(S), _t(E), mode)
        _equal(a2, a4, f"n={n} {mode}")
        got = a4[key].cpu().numpy().astype(np.int64)
        want = ref["count"] if mode == "count" else (ref["count"] > 0)
        assert np.array_equal(got[ok], want[ok].astype(np.int64)), (n, mode)
    mesh.close()


def test_wide_oracle_parity_config1_full():
    w = wl.config1()
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32), leaf_size=4)
    mesh.set_opts(branching=4)
    got = mesh.query(_t(w.S), _t(w.E), "bool|first")
    torch.cuda.synchronize()
    ref = parity.oracle_reference(w.V, w.T, w.S, w.E)
    rep = parity.compare(ref, {k: v.cpu().numpy() for k, v in got.items()}, {"bool", "first"})
    parity.assert_parity(rep)
    mesh.close()


def test_wide_after_refit_and_rebuild():
    w = wl.config4(n_r=200_000)
    V, T = _t(w.V), _t(w.T, torch.int32)
    S, E = _t(w.S), _t(w.E)
    mesh = rsi.Mesh(V, T, branching=4)
    assert mesh.opts()["branching"] == 4
    V2 = V.clone()
    V2[:, 2] += 0.05 * torch.sin(7 * V2[:, 0])
    mesh.refit(V2)
    r4 = mesh.query(S, E, "first")
    fresh = rsi.Mesh(V2, T)
    r2 = fresh.query(S, E, "first")
    torch.cuda.synchronize()
    _equal(r2, r4, "refit")
    mesh.rebuild(V, T)
    r4b = mesh.query(S, E, "first")
    fresh.rebuild(V, T)
    r2b = fresh.query(S, E, "first")
    torch.cuda.synchronize()
    _equal(r2b, r4b, "rebuild")
    mesh.close()
    fresh.close()


def test_wide_batch_and_graph():
    ws = wl.config5(n_meshes=8, tri_lo=500, tri_hi=20_000, seg_lo=2_000, seg_hi=30_000, seed=321)
    meshes = [(_t(w.V), _t(w.T, torch.int32)) for w in ws]
    segs = [(_t(w.S), _t(w.E)) for w in ws]
    b = rsi.Batch(meshes)
    ref = b.query(segs, "bool|first")
    b.set_opts(branching=4)
    got = b.query(segs, "bool|first")
    torch.cuda.synchronize()
    for k in range(len(ws)):
        _equal(ref[k], got[k], ws[k].name)
    outs = b.alloc_outputs(segs, "bool|first")
    b.capture(segs, "bool|first", outs, rebuild=True)
    for _ in range(3):
        b.replay()
        torch.cuda.synchronize()
        for k in range(len(ws)):
            _equal(ref[k], outs[k], "graph-" + ws[k].name)
        b.query(segs, "bool")  # eager work between replays
    b.close()


def test_branching_option_validation():
    w = wl.config1(n_r=100)
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    with pytest.raises(rsi.RsiError):
        mesh.set_opts(branching=3)
    assert mesh.opts()["branching"] == 4  # the default is kept
    mesh.close()


@pytest.mark.parametrize("offset,size", [(2.0 ** 35, 2.0 ** 20), (-(2.0 ** 30), 2.0 ** 22)])
def test_wide_far_from_origin_matches_oracle(offset, size):
    """A mesh far from the coordinate origin (2^35 or -2^30 away, 2^20 or
    2^22 across, so FP32 still resolves it): corner offsets are large next
    to the node boxes, and so are the rounding margins.  Both walks must
    meet the FP64 oracle on every non-degenerate segment (bit-identity
    between them is not required here: on such coarse FP32 coordinates the
    looser quantised boxes may let a triangle test that sits within rounding
    of its decision run where the binary walk culls it)."""
    w = wl.config1(n_r=4000)
    move = lambda a: (a.astype(np.float64) * size + offset).astype(np.float32)
    Vh, Sh, Eh = move(w.V), move(w.S), move(w.E)
    ref = parity.oracle_reference(Vh, w.T, Sh, Eh, cap=4)
    V, T = _t(Vh), _t(w.T, torch.int32)
    S, E = _t(Sh), _t(Eh)
    for br in (2, 4):
        mesh = rsi.Mesh(V, T, branching=br)
        out = mesh.query(S, E, "bool|first|all", capacity=4)
        torch.cuda.synchronize()
        rep = parity.compare(ref, out, {"bool", "first", "all"}, cap=4)
        assert rep["hits"] > 50, rep
        # the hit point is stored in FP32, whose spacing at these magnitudes
        # exceeds the usual 1e-5 L: check it against that spacing instead
        p_bad = rep.pop("first_p_bad")
        parity.assert_parity(rep)
        if p_bad:
            ok = (ref["degenerate"] == 0) & (ref["first_tri"] >= 0)
            P = out["point"].cpu().numpy().astype(np.float64)[ok]
            Pr = ref["first_p"][ok]
            tol = parity.T_TOL * ref["extent"] + 2.0 ** -23 * np.abs(Pr)
            assert np.all(np.abs(P - Pr) <= tol), br
        mesh.close()
