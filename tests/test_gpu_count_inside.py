"""GPU parity of the crossing-count mode and the odd-parity inside test.

RSI_COUNT is the paper's `intercept_count` output (Section 2.4): the exact
number of crossings per segment with no list; its odd parity along a
segment from a point to outside a closed surface tells whether the point is
inside (Section 2.6).  Both go through the C ABI and are compared with the
FP64 oracle (counts bit-exact on non-degenerate segments) and, for the
inside test on star-shaped meshes, with regions known in closed form.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl
import oracle
from tests import parity
from tests.test_oracle_inside import star_regions

pytestmark = pytest.mark.gpu

DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


@pytest.mark.parametrize("mode", ["count", "count|bool", "count|first", "count|first|bool"])
def test_count_mode_config1_full(mode):
    w = wl.config1()
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    out = mesh.query(_t(w.S), _t(w.E), mode)
    torch.cuda.synchronize()
    ref = parity.oracle_reference(w.V, w.T, w.S, w.E)
    ok = ref["degenerate"] == 0
    cnt = out["count"].cpu().numpy()
    assert np.array_equal(cnt[ok], ref["count"][ok])
    modes = [m for m in ("bool", "first") if m in mode]
    if modes:
        rep = parity.compare(ref, out, modes)
        bad = {k: v for k, v in rep.items() if k.endswith(("_mismatch", "_bad")) and v}
        assert not bad, rep
    mesh.close()


def test_count_mode_matches_all_hits_on_closed_sphere():
    """Counts of the count-only pass equal the all-hits pass's exact counts,
    on 1M segments against the 499,280-triangle closed sphere."""
    w = wl.config3(n_r=1_000_000)
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    S, E = _t(w.S), _t(w.E)
    c = mesh.query(S, E, "count")["count"]
    a = mesh.query(S, E, "all", capacity=4)["count"]
    torch.cuda.synchronize()
    assert torch.equal(c, a)
    # sampled against the oracle
    sel = wl.subset(w.n_r, 2000, wl.seed_for(3, 5))
    ref = parity.oracle_reference(w.V, w.T, w.S[sel], w.E[sel])
    ok = ref["degenerate"] == 0
    assert np.array_equal(c.cpu().numpy()[sel][ok], ref["count"][ok])
    mesh.close()


def test_inside_small_sphere_full_oracle():
    V, T = wl.noisy_sphere(20, 123, 0.3)
    V = V.astype(np.float32)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    rng = np.random.default_rng(wl.seed_for(6, 2))
    lo, hi = wl.mesh_bbox(V)
    c, h = 0.5 * (lo + hi), 0.75 * (hi - lo)
    P = rng.uniform(c - h, c + h, (50_000, 3)).astype(np.float32)
    out = mesh.inside(_t(P))
    torch.cuda.synchronize()
    E = out["E"].cpu().numpy()
    # the far ends follow the documented rule (FP32 rounding aside)
    U = np.array([0.6, 0.41, 0.91]) / np.linalg.norm([0.6, 0.41, 0.91])
    lo64, hi64 = lo.astype(np.float64), hi.astype(np.float64)
    L = np.linalg.norm(P - 0.5 * (lo64 + hi64), axis=1) + np.linalg.norm(hi64 - lo64) + 1
    assert np.allclose(E, P + L[:, None] * U, rtol=0, atol=1e-5 * L.max())
    ref = parity.oracle_reference(V, T, P, E)
    ok = ref["degenerate"] == 0
    assert ok.mean() > 0.99
    cnt = out["count"].cpu().numpy()
    ins = out["inside"].cpu().numpy()
    assert np.array_equal(cnt[ok], ref["count"][ok])
    assert np.array_equal(ins, (cnt & 1).astype(np.uint8))
    # closed-form regions of the star-shaped surface
    r_in, r_out = star_regions(V, T)
    r = np.linalg.norm(P.astype(np.float64), axis=1)
    assert np.all(ins[r < 0.999 * r_in] == 1)
    assert np.all(ins[r > 1.001 * r_out] == 0)
    mesh.close()


def test_inside_config3_mesh_two_million_points():
    """Full size: the 499,280-triangle sphere, 2M points uniform in 1.5x its
    box; every point in the closed-form regions is classified exactly, and a
    seeded sample matches the oracle."""
    V, T = wl.config3_mesh(158)
    V = V.astype(np.float32)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    P = wl.inside_points(V, 2_000_000, wl.seed_for(6, 3))
    out = mesh.inside(_t(P))
    torch.cuda.synchronize()
    ins = out["inside"].cpu().numpy()
    r_in, r_out = star_regions(V, T)
    r = np.linalg.norm(P.astype(np.float64), axis=1)
    inner, outer = r < 0.999 * r_in, r > 1.001 * r_out
    assert inner.sum() > 10_000 and outer.sum() > 10_000
    # FP32 Moller-Trumbore is not watertight: a segment through a shared edge
    # or vertex can be counted twice or not at all.  Every point whose parity
    # disagrees with the closed form must be such a degenerate case.
    wrong = np.nonzero((inner & (ins == 0)) | (outer & (ins == 1)))[0]
    assert wrong.size <= 1e-4 * P.shape[0]
    if wrong.size:
        Ew = out["E"].cpu().numpy()[wrong]
        L = float(np.linalg.norm(V.max(0) - V.min(0)))
        deg = oracle.degenerate(V, T, P[wrong], Ew, 1e-6 * L)
        assert np.all(deg != 0), wrong[deg == 0]
    sel = wl.subset(P.shape[0], 1000, wl.seed_for(6, 4))
    E = out["E"].cpu().numpy()[sel]
    ref = parity.oracle_reference(V, T, P[sel], E)
    ok = ref["degenerate"] == 0
    cnt = out["count"].cpu().numpy()[sel]
    assert np.array_equal(cnt[ok], ref["count"][ok])
    mesh.close()


def test_inside_edge_cases():
    V, T = wl.noisy_sphere(4, 5, 0.3)
    mesh = rsi.Mesh(_t(V.astype(np.float32)), _t(T, torch.int32))
    empty = mesh.inside(torch.zeros((0, 3), dtype=torch.float32, device=DEV))
    assert empty["inside"].numel() == 0
    with pytest.raises(rsi.RsiError):
        rsi.rsi_inside(mesh.handle, _t(np.zeros((4, 3))), None)
    mesh.close()
    # no triangles: every point is outside
    m0 = rsi.Mesh(_t(np.zeros((3, 3))), torch.zeros((0, 3), dtype=torch.int32, device=DEV))
    out = m0.inside(_t(np.random.default_rng(1).uniform(-1, 1, (1000, 3))))
    torch.cuda.synchronize()
    assert int(out["inside"].sum()) == 0 and int(out["count"].abs().sum()) == 0
    m0.close()
