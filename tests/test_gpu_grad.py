"""GPU adjoint of the first hit (differentiable form of the paper's
`barycentric` output, Section 2.4) against the FP64 oracle gradient and
FP64 central finite differences.

Tolerances: dS and dE per segment within 1e-5 relative (plus a 1e-7 floor of
the largest magnitude); dV per element within 1e-5 of the sum of absolute
contributions to that element (contributions of opposite sign cancel), and
within 1e-5 relative in 2-norm over the whole vector.  The device sums the
contributions without atomics in a fixed order, so repeated calls must give
the same bits.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl
import oracle
from tests import parity

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def _check_dv(dv_gpu, dv_ref, dv_abs, rel=1e-5):
    err = np.abs(dv_gpu - dv_ref)
    bad = err > rel * dv_abs + 1e-30
    assert not bad.any(), f"{bad.sum()} dV elements off; worst ratio {np.max(err / (dv_abs + 1e-30)):.3g}"
    norm = np.linalg.norm(dv_gpu - dv_ref) / np.linalg.norm(dv_ref)
    assert norm <= rel, norm


def _check_seg(g_gpu, g_ref, rel=1e-5):
    floor = 1e-7 * np.abs(g_ref).max()
    bad = np.abs(g_gpu - g_ref) > rel * np.abs(g_ref) + floor
    assert not bad.any(), f"{bad.sum()} per-segment gradient values off"


@pytest.mark.parametrize("n_half", [30_000, 120_000])
def test_adjoint_matches_oracle_random_upstream(n_half):
    """60k and 240k segments (about one and four per triangle: cells with
    few and with many records each)."""
    V, T = wl.noise_heightfield(60, 17, 0.2)
    rng = np.random.default_rng(3)
    S1, E1 = wl.segments_near_vertical(rng, n_half)
    S2, E2 = wl.segments_random_dir(rng, V.min(0), V.max(0), n_half)
    S = np.concatenate([S1, S2])
    E = np.concatenate([E1, E2])
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    out = mesh.query(_t(S), _t(E), "first")
    ref = parity.oracle_reference(V, T, S, E)
    tri = out["tri"].cpu().numpy()
    ok = (ref["degenerate"] == 0) & (tri == ref["first_tri"]) & (tri >= 0)
    assert ok.sum() > n_half
    n = S.shape[0]
    g_t = (rng.standard_normal(n) * ok).astype(np.float32)
    g_uv = (rng.standard_normal((n, 2)) * ok[:, None]).astype(np.float32)
    g_p = (rng.standard_normal((n, 3)) * ok[:, None]).astype(np.float32)
    tri_in = np.where(ok, tri, -1).astype(np.int32)
    dV, dS, dE = mesh.first_hit_backward(_t(V), _t(S), _t(E), _t(tri_in, torch.int32), _t(g_t), _t(g_uv),
                                         _t(g_p))
    torch.cuda.synchronize()
    rV, rS, rE, rabs = oracle.first_hit_grad(V, T, S, E, tri_in, ref["first_tuv"], g_t, g_uv, g_p,
                                             with_abs=True)
    _check_dv(dV.cpu().numpy().astype(np.float64), rV, rabs)
    # a second call on the same inputs (the handle's scratch now reused)
    # gives the same bits: the sums run in a fixed order, without atomics
    dV2, dS2, dE2 = mesh.first_hit_backward(_t(V), _t(S), _t(E), _t(tri_in, torch.int32), _t(g_t), _t(g_uv),
                                            _t(g_p))
    torch.cuda.synchronize()
    assert torch.equal(dV, dV2) and torch.equal(dS, dS2) and torch.equal(dE, dE2)
    _check_seg(dS.cpu().numpy()[ok].astype(np.float64), rS[ok])
    _check_seg(dE.cpu().numpy()[ok].astype(np.float64), rE[ok])
    assert not dS.cpu().numpy()[~ok].any() and not dE.cpu().numpy()[~ok].any()


def test_autograd_function_matches_direct_call():
    V, T = wl.noise_heightfield(40, 5, 0.2)
    rng = np.random.default_rng(9)
    S, E = wl.segments_near_vertical(rng, 20_000)
    Vt = _t(V).requires_grad_(True)
    St = _t(S).requires_grad_(True)
    Et = _t(E).requires_grad_(True)
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    t, uv, P, tri = rsi.FirstHit.apply(Vt, St, Et, mesh)
    loss = (P[:, 2] ** 2).sum() + t.sum() + uv.sum()
    loss.backward()
    g_p = torch.zeros_like(P)
    g_p[:, 2] = 2 * P[:, 2].detach()
    dV, dS, dE = mesh.first_hit_backward(_t(V), _t(S), _t(E), tri, torch.ones_like(t), torch.ones_like(uv), g_p)
    scale = dV.abs().max()
    assert torch.allclose(Vt.grad, dV, atol=1e-6 * float(scale), rtol=1e-5)
    assert torch.allclose(St.grad, dS) and torch.allclose(Et.grad, dE)


def test_c4_fwd_bwd_against_oracle_and_finite_differences():
    """Differentiable first hit on the 317 x 317 heightfield (199,712
    triangles) with 4M near-vertical segments and loss
    L = sum (P_z - g(x_S, y_S))^2 for a second seeded surface g.  The check
    set is a seeded 100k sample plus every segment that can hit a triangle
    around one of 64 sampled interior vertices; the loss is masked to it."""
    n = 317
    w = wl.config4()
    Vg, _ = wl.config4_target(n)
    V, T, S, E = w.V, w.T, w.S, w.E
    gz = Vg[:, 2].astype(np.float64)

    # g(x, y): bilinear interpolation of the target grid's vertex heights
    def target_at(x, y):
        X = np.clip(x * (n - 1), 0, n - 1 - 1e-9)
        Y = np.clip(y * (n - 1), 0, n - 1 - 1e-9)
        i = X.astype(np.int64)
        j = Y.astype(np.int64)
        a, b = X - i, Y - j
        k = j * n + i
        return (gz[k] * (1 - a) * (1 - b) + gz[k + 1] * a * (1 - b) + gz[k + n] * (1 - a) * b
                + gz[k + n + 1] * a * b)
    target = target_at(S[:, 0].astype(np.float64), S[:, 1].astype(np.float64)).astype(np.float32)

    rng = np.random.default_rng(wl.seed_for(4, 3))
    # 64 interior vertices and the segments whose xy box meets their 1-ring box
    vi = rng.integers(2, n - 2, size=(64, 2))
    fd_vertices = vi[:, 1] * n + vi[:, 0]
    ring_lo = np.stack([(vi[:, 0] - 1) / (n - 1), (vi[:, 1] - 1) / (n - 1)], 1)
    ring_hi = np.stack([(vi[:, 0] + 1) / (n - 1), (vi[:, 1] + 1) / (n - 1)], 1)
    seg_lo = np.minimum(S[:, :2], E[:, :2])
    seg_hi = np.maximum(S[:, :2], E[:, :2])
    near = np.zeros(S.shape[0], bool)
    for k in range(64):
        near |= np.all((seg_hi >= ring_lo[k]) & (seg_lo <= ring_hi[k]), axis=1)
    chk = np.union1d(wl.subset(S.shape[0], 100_000, wl.seed_for(4, 3)), np.nonzero(near)[0])

    # GPU forward + backward with the loss masked to the check set
    mesh = rsi.Mesh(_t(V), _t(T, torch.int32))
    Vt = _t(V)
    St, Et = _t(S), _t(E)
    t, uv, P, tri = rsi.FirstHit.apply(Vt, St, Et, mesh)
    mask = torch.zeros(S.shape[0], dtype=torch.float32, device=DEV)
    mask[_t(chk, torch.int64)] = 1.0
    resid = P[:, 2] - _t(target)
    g_p = torch.zeros_like(P)
    g_p[:, 2] = 2 * resid * mask
    dV, dS, dE = mesh.first_hit_backward(Vt, St, Et, tri, None, None, g_p.contiguous())
    torch.cuda.synchronize()

    # oracle on the check set
    Sc, Ec = S[chk], E[chk]
    ref = parity.oracle_reference(V, T, Sc, Ec)
    tri_c = tri.cpu().numpy()[chk]
    clean = ref["degenerate"] == 0
    # on the regular grid about 3 edge lines per cell width lie within the
    # 1e-6 * L band, so a few tenths of a percent are near-degenerate
    assert clean.mean() > 0.99
    assert int((clean & (ref["first_tri"] != tri_c)).sum()) == 0
    ok = clean
    assert np.all(ref["count"][ok] == 1)
    # the GPU's masked loss must skip the same (degenerate) segments
    drop = chk[~ok]
    if drop.size:
        g_p[_t(drop, torch.int64)] = 0
        dV, dS, dE = mesh.first_hit_backward(Vt, St, Et, tri, None, None, g_p.contiguous())
    # the same call again: identical bits (fixed summation order, no atomics)
    dV_again, _, _ = mesh.first_hit_backward(Vt, St, Et, tri, None, None, g_p.contiguous())
    assert torch.equal(dV, dV_again)
    dVn = dV.cpu().numpy().astype(np.float64)
    tri_ok = np.where(ok, tri_c, -1)
    # (a) the adjoint alone: the oracle differentiates with the same upstream
    # gradient the GPU used (formed from the GPU's FP32 hit points)
    gp_gpu = g_p.cpu().numpy()[chk].astype(np.float64)
    aV, aS, aE, aabs = oracle.first_hit_grad(V, T, Sc, Ec, tri_ok, ref["first_tuv"], g_p=gp_gpu, with_abs=True)
    _check_dv(dVn, aV, aabs)
    _check_seg(dS.cpu().numpy()[chk][ok].astype(np.float64), aS[ok])
    _check_seg(dE.cpu().numpy()[chk][ok].astype(np.float64), aE[ok])
    # (b) end to end: the oracle's own FP64 hit points form its loss gradient
    gp_ref = np.zeros((chk.size, 3))
    gp_ref[:, 2] = 2 * (ref["first_p"][:, 2] - target[chk])
    gp_ref[~ok] = 0.0
    rV, rS, rE = oracle.first_hit_grad(V, T, Sc, Ec, tri_ok, ref["first_tuv"], g_p=gp_ref)
    rel = np.linalg.norm(dVn - rV) / np.linalg.norm(rV)
    print(f"end-to-end dL/dV relative error (2-norm): {rel:.3g}")
    assert rel <= 1e-5
    dSc = dS.cpu().numpy()[chk].astype(np.float64)
    assert np.linalg.norm(dSc - rS) / np.linalg.norm(rS) <= 1e-5

    # central differences (FP64, h = 1e-4) of the masked loss in each sampled
    # vertex's z, over the check segments that stay clear of every edge
    u, v = ref["first_tuv"][:, 1], ref["first_tuv"][:, 2]
    clear = ok & (np.minimum(np.minimum(u, v), 1 - u - v) > 1e-3)
    V64 = V.astype(np.float64)
    h = 1e-4
    n_checked = 0
    for k in fd_vertices:
        inc = np.any(T[np.where(clear, tri_c, 0)] == k, axis=1) & clear
        if not inc.any():
            continue
        # the GPU gradient of the loss restricted to `clear` segments
        sel = chk[inc]
        # upstream from the oracle's FP64 residuals, as in the differenced loss
        g_k = torch.zeros_like(P)
        g_k[_t(sel, torch.int64), 2] = _t(2 * (ref["first_p"][inc, 2] - target[sel].astype(np.float64)))
        dVk, _, _ = mesh.first_hit_backward(Vt, St, Et, tri, None, None, g_k.contiguous())
        gpu = float(dVk[int(k), 2])
        losses = []
        for sgn in (1, -1):
            Vp = V64.copy()
            Vp[k, 2] += sgn * h
            r = oracle.query(Vp, T, Sc[inc], Ec[inc])
            assert np.array_equal(r["first_tri"], tri_c[inc])
            losses.append(np.sum((r["first_p"][:, 2] - target[sel].astype(np.float64)) ** 2))
        fd = (losses[0] - losses[1]) / (2 * h)
        gp_k = np.zeros((chk.size, 3))
        gp_k[inc, 2] = 2 * (ref["first_p"][inc, 2] - target[sel])
        _, _, _, abs_k = oracle.first_hit_grad(V, T, Sc, Ec, np.where(inc, tri_c, -1), ref["first_tuv"],
                                               g_p=gp_k, with_abs=True)
        assert abs(gpu - fd) <= 1e-5 * abs_k[k, 2] + 1e-9, (int(k), gpu, fd, abs_k[k, 2])
        n_checked += 1
    assert n_checked >= 60


def test_gradient_bits_independent_of_tree_options():
    """The backward reads the hit triangles' records by sorted position and
    sums in a fixed order over cells of sorted positions, so the leaf size
    and the walk (binary or four-way) that produced the same first hits
    must give the same dV, dS and dE bits."""
    V, T = wl.noise_heightfield(60, 17, 0.2)
    rng = np.random.default_rng(9)
    S, E = wl.segments_near_vertical(rng, 100_000)
    Vt, Tt, St, Et = _t(V), _t(T, torch.int32), _t(S), _t(E)
    g = torch.zeros(S.shape[0], 3, device=DEV)
    g[:, 2] = 1.0
    base = None
    for leaf, branching in ((1, 4), (4, 4), (1, 2), (8, 2)):
        mesh = rsi.Mesh(Vt, Tt, leaf_size=leaf, branching=branching)
        out = mesh.query(St, Et, "first")
        dV, dS, dE = rsi.rsi_first_hit_backward(mesh.handle, Vt, St, Et, out["tri"], None, None, g)
        torch.cuda.synchronize()
        got = (out["tri"].cpu(), dV.cpu(), dS.cpu(), dE.cpu())
        mesh.close()
        if base is None:
            base = got
            assert int((got[0] >= 0).sum()) > 50_000
        else:
            for a, b in zip(base, got):
                assert torch.equal(a, b), (leaf, branching)
