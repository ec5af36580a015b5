"""CPU model of the first-hit adjoint's data flow (no GPU): the order in
which the device groups and sums the vertex contributions, restated in numpy
and checked against the FP64 oracle's gradient.

The device kernels (adjoint.hip) solve every segment in input order, group
the (hit triangle's Morton position, segment) pairs by cells of 1,024
positions with a stable pass, cut each cell's pairs into four consecutive
quarters, and in each quarter walk the pairs tile by tile (1,024 pairs),
rank the tile's pairs stably by (position mod 256) and add each triangle's
records in that order in FP64; the four quarters' sums are then added in
order, and finally the (triangle, corner) terms of each vertex from a table
sorted by vertex.  No atomic operation is involved, so the only ways to lose
a contribution would be a wrong grouping or a wrong range; this model walks
exactly those ranges (including cells that span several tiles, empty cells,
misses and the last, partly filled cell) and must reproduce the oracle's
gradient.
"""
import numpy as np

import oracle
from paper_2209_02878_amd import workloads as wl

CELL_BITS, TILE, CHUNKS = 10, 512, 4


def _model(V, T, S, E, tri, g_p, rank, corner0="fp64"):
    """dV as the device forms it.  The record holds lambda and the corner
    weights rounded to FP32; corner0="fp64" rounds 1 - u - v from its FP64
    value (the device's record), corner0="from_uv" forms it from the rounded
    u and v instead (shown below to lose accuracy near the edge v1 v2)."""
    n_t, n_r = T.shape[0], S.shape[0]
    # k_adj_solve: per segment, lambda and the corner weights (FP32), the
    # key (sorted position or n_t)
    keys = np.full(n_r, n_t, np.int64)
    rec = np.zeros((n_r, 6))
    for i in range(n_r):
        j = tri[i]
        if j < 0:
            continue
        v0, v1, v2 = (V[T[j, c]].astype(np.float64) for c in range(3))
        s, e = S[i].astype(np.float64), E[i].astype(np.float64)
        d = e - s
        M = np.stack([-d, v1 - v0, v2 - v0], 1)
        if np.linalg.det(M) == 0:
            continue
        t, u, v = np.linalg.solve(M, s - v0)
        tb = g_p[i] @ d
        lam = np.linalg.solve(M.T, np.array([tb, 0.0, 0.0]))
        f = lambda x: float(np.float32(x))
        w0 = f(1.0 - u - v) if corner0 == "fp64" else 1.0 - f(u) - f(v)
        rec[i] = [f(lam[0]), f(lam[1]), f(lam[2]), w0, f(u), f(v)]
        keys[i] = rank[j]
    # stable grouping by cell
    order = np.argsort(keys >> CELL_BITS, kind="stable")
    sk = keys[order]
    n_cells = (n_t + (1 << CELL_BITS) - 1) >> CELL_BITS
    tri_sum = np.zeros((n_t, 3, 3))
    for g in range(n_cells):
        clo = np.searchsorted(sk >> CELL_BITS, g, side="left")
        chi = np.searchsorted(sk >> CELL_BITS, g + 1, side="left")
        parts = []
        for c in range(CHUNKS):
            lo, hi = clo + (chi - clo) * c // CHUNKS, clo + (chi - clo) * (c + 1) // CHUNKS
            acc = np.zeros((1 << CELL_BITS, 3, 3))
            for c0 in range(lo, hi, TILE):
                ks = sk[c0:min(c0 + TILE, hi)]
                segs = order[c0:min(c0 + TILE, hi)]
                sel = ks < n_t
                local = ks[sel] & ((1 << CELL_BITS) - 1)
                # stable rank by (local mod 256) within the tile; each
                # thread then adds its records in that order
                for p in np.argsort(local & 255, kind="stable"):
                    r = rec[segs[sel][p]]
                    lam, w = r[:3], -r[3:6]
                    acc[local[p]] += w[:, None] * lam[None, :]
            parts.append(acc)
        total = np.zeros((1 << CELL_BITS, 3, 3))
        for acc in parts:  # the quarters in order
            total += acc
        base = g << CELL_BITS
        m = min(1 << CELL_BITS, n_t - base)
        tri_sum[base:base + m] = total[:m]
    # vertex incidence table sorted by vertex (stable): (vertex, 3 * position + corner)
    inc_v = T.reshape(-1)
    inc_tc = 3 * np.repeat(rank, 3) + np.tile(np.arange(3), n_t)
    o = np.argsort(inc_v, kind="stable")
    dV = np.zeros((V.shape[0], 3))
    for v, tc in zip(inc_v[o], inc_tc[o]):
        dV[v] += tri_sum[tc // 3, tc % 3]
    return dV


def test_adjoint_grouping_model_matches_oracle_gradient():
    # 2,888 triangles: three cells, the last one partly filled; segments in
    # random order, some missing the mesh; cells span several tiles
    V, T = wl.noise_heightfield(39, 11, 0.2)
    n_t = T.shape[0]
    rng = np.random.default_rng(4)
    S, E = wl.segments_near_vertical(rng, 6000)
    S[:300, :2] += 2.0  # misses
    E[:300, :2] += 2.0
    ref = oracle.query(V, T, S, E)
    tri = ref["first_tri"]
    assert (tri < 0).sum() >= 300 and (tri >= 0).sum() > 5000
    # any permutation serves as the Morton order of the triangles
    rank = rng.permutation(n_t).astype(np.int64)
    g_p = np.zeros((S.shape[0], 3))
    g_p[:, 2] = rng.standard_normal(S.shape[0])
    dV = _model(V, T, S, E, tri, g_p, rank)
    rV, _, _, rabs = oracle.first_hit_grad(V, T, S, E, tri, ref["first_tuv"], g_p=g_p, with_abs=True)
    # the device's bar: within 1e-5 of the sum of absolute contributions
    assert np.all(np.abs(dV - rV) <= 1e-5 * rabs + 1e-30)
    assert np.abs(dV - rV).max() <= 1e-6 * np.abs(rV).max()
    assert np.count_nonzero(rV) > 0


def test_corner_weight_rounding_near_an_edge():
    """Hits close to the edge v1 v2 give vertex v0 only small weights
    1 - u - v.  Formed from u and v already rounded to FP32, that weight keeps
    an absolute error of a few 1e-8, which is then a large share of the small
    sum of |contributions| at v0 and breaks the per-element bar; rounded from
    its FP64 value it keeps FP32 relative accuracy and meets it."""
    V = np.array([[0.1, 0.2, 0.0], [1.3, 0.1, 0.05], [0.15, 1.1, -0.03]], np.float32)
    T = np.array([[0, 1, 2]], np.int32)
    rng = np.random.default_rng(9)
    n = 8
    # vertical segments through points with 1 - u - v in [1e-5, 1e-4]
    w0 = rng.uniform(1e-5, 1e-4, n)
    u = rng.uniform(0.2, 0.8, n) * (1.0 - w0)
    v = 1.0 - w0 - u
    Vd = V.astype(np.float64)
    xy = (w0[:, None] * Vd[0] + u[:, None] * Vd[1] + v[:, None] * Vd[2])[:, :2]
    S = np.concatenate([xy, np.full((n, 1), 1.0)], 1).astype(np.float32)
    E = np.concatenate([xy, np.full((n, 1), -1.0)], 1).astype(np.float32)
    ref = oracle.query(V, T, S, E)
    tri = ref["first_tri"]
    assert np.all(tri == 0)
    g_p = np.zeros((n, 3))
    g_p[:, 2] = 1.0
    rV, _, _, rabs = oracle.first_hit_grad(V, T, S, E, tri, ref["first_tuv"], g_p=g_p, with_abs=True)
    rank = np.zeros(1, np.int64)
    good = _model(V, T, S, E, tri, g_p, rank, corner0="fp64")
    bad = _model(V, T, S, E, tri, g_p, rank, corner0="from_uv")
    ratio = lambda d: np.max(np.abs(d - rV) / (rabs + 1e-30))
    assert ratio(good) <= 1e-6
    assert ratio(bad) > 1e-5
