"""Pins of the oracle's first-hit gradient.

The gradient differentiates the first hit (t, u, v, P) of each segment with
respect to the vertices and both segment ends.  It is pinned by
* a closed form: for a vertical segment over a heightfield the hit height is
  the barycentric blend of the three vertex heights, so d(P_z)/d(z_k) is the
  barycentric weight of vertex k and moving either end vertically leaves P_z
  unchanged;
* central finite differences of the oracle's FP64 forward query, which is
  itself pinned in test_oracle_pins.py.
"""
import numpy as np

import oracle
from paper_2209_02878_amd import workloads as wl


def test_vertical_hit_height_gradient_is_barycentric():
    n = 24
    V, T = wl.noise_heightfield(n, 77, 0.2)
    rng = np.random.default_rng(8)
    m = 500
    xy = rng.uniform(0.01, 0.99, size=(m, 2))
    S = np.concatenate([xy, np.full((m, 1), 1.0)], 1)
    E = np.concatenate([xy, np.full((m, 1), -1.0)], 1)
    r = oracle.query(V, T, S, E)
    assert np.all(r["count"] == 1)
    g_p = np.zeros((m, 3))
    g_p[:, 2] = 1.0
    dV, dS, dE, dV_abs = oracle.first_hit_grad(V, T, S, E, r["first_tri"], r["first_tuv"], g_p=g_p,
                                               with_abs=True)
    # expected: scatter the barycentric weights (1-u-v, u, v) into z
    t, u, v = r["first_tuv"].T
    want = np.zeros(V.shape[0])
    tri = T[r["first_tri"]]
    np.add.at(want, tri[:, 0], 1 - u - v)
    np.add.at(want, tri[:, 1], u)
    np.add.at(want, tri[:, 2], v)
    np.testing.assert_allclose(dV[:, 2], want, atol=1e-12)
    # every contribution to a z component is a nonnegative weight here
    np.testing.assert_allclose(dV_abs[:, 2], want, atol=1e-12)
    np.testing.assert_allclose(dS[:, 2], 0.0, atol=1e-12)
    np.testing.assert_allclose(dE[:, 2], 0.0, atol=1e-12)


def _loss(r, w):
    tuv = r["first_tuv"]
    return float(np.sum(w["t"] * tuv[:, 0]) + np.sum(w["uv"] * tuv[:, 1:]) + np.sum(w["p"] * r["first_p"]))


def test_gradient_matches_central_differences():
    V, T = wl.noisy_sphere(6, 31, 0.3)
    V = V.astype(np.float64)
    rng = np.random.default_rng(12)
    S, E = wl.segments_in_box(rng, V.min(0), V.max(0), 400, scale=1.5)
    S = S.astype(np.float64)
    E = E.astype(np.float64)
    base = oracle.query(V, T, S, E)
    flags = oracle.degenerate(V, T, S, E, delta=1e-4)
    # keep clean hits: away from edges and not grazing (the FD truncation term
    # grows like 1/sin^3 of the angle between segment and triangle)
    hit = base["count"] > 0
    tri = T[np.where(hit, base["first_tri"], 0)]
    nrm = np.cross(V[tri[:, 1]] - V[tri[:, 0]], V[tri[:, 2]] - V[tri[:, 0]])
    d = E - S
    sin = np.abs(np.sum(nrm * d, 1)) / (np.linalg.norm(nrm, axis=1) * np.linalg.norm(d, axis=1))
    keep = hit & (flags == 0) & (sin > 0.2)
    S, E = S[keep], E[keep]
    base = oracle.query(V, T, S, E)
    m = S.shape[0]
    assert m > 100
    w = {"t": rng.standard_normal(m), "uv": rng.standard_normal((m, 2)), "p": rng.standard_normal((m, 3))}
    dV, dS, dE = oracle.first_hit_grad(V, T, S, E, base["first_tri"], base["first_tuv"],
                                       g_t=w["t"], g_uv=w["uv"], g_p=w["p"])
    h = 1e-6
    for trial in range(6):
        pV = rng.standard_normal(V.shape)
        pS = rng.standard_normal(S.shape)
        pE = rng.standard_normal(E.shape)
        if trial % 3 == 1:
            pS[:] = 0
            pE[:] = 0
        elif trial % 3 == 2:
            pV[:] = 0
        rp = oracle.query(V + h * pV, T, S + h * pS, E + h * pE)
        rm = oracle.query(V - h * pV, T, S - h * pS, E - h * pE)
        assert np.array_equal(rp["first_tri"], base["first_tri"])
        assert np.array_equal(rm["first_tri"], base["first_tri"])
        fd = (_loss(rp, w) - _loss(rm, w)) / (2 * h)
        an = float(np.sum(dV * pV) + np.sum(dS * pS) + np.sum(dE * pE))
        assert abs(fd - an) <= 1e-6 * max(1.0, abs(an)), (trial, fd, an)


def test_miss_contributes_nothing():
    V = np.array([[0, 0, 0], [1, 0, 0], [0, 1, 0]], np.float64)
    T = np.array([[0, 1, 2]], np.int32)
    S = np.array([[2.0, 2.0, 1.0]])
    E = np.array([[2.0, 2.0, -1.0]])
    r = oracle.query(V, T, S, E)
    assert r["first_tri"][0] == -1
    dV, dS, dE = oracle.first_hit_grad(V, T, S, E, r["first_tri"], np.zeros((1, 3)),
                                       g_t=np.ones(1), g_p=np.ones((1, 3)))
    assert not dV.any() and not dS.any() and not dE.any()
