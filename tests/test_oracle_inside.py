"""Pins of the odd-parity inside test on the oracle side (CPU).

The paper counts the crossings of a segment (Section 2.4, extended usage)
and notes that an odd count puts the segment's start point inside a closed
surface (Section 2.6).
On a closed star-shaped mesh two regions are known without any crossing
arithmetic: points closer to the centre than every triangle's plane are
inside (the ray from the centre meets the surface where it lies on some
triangle plane), and points beyond the largest vertex radius are outside.
The oracle's crossing counts along the library's inside-test segments must
give the same parity there.
"""
import numpy as np

import oracle
from paper_2209_02878_amd import workloads as wl

# the documented inside-test segment: from P along u to P + L u,
# L = |P - c| + 2 R + 1 (c, R: centre and half diagonal of the mesh box)
U = np.array([0.6, 0.41, 0.91]) / np.linalg.norm([0.6, 0.41, 0.91])


def far_ends(V, P):
    lo, hi = V.min(0), V.max(0)
    c, R = 0.5 * (lo + hi), 0.5 * np.linalg.norm(hi - lo)
    L = np.linalg.norm(P - c, axis=1) + 2 * R + 1
    return (P + L[:, None] * U).astype(np.float32)


def star_regions(V, T):
    """Inner radius (min distance from the origin to a triangle plane) and
    outer radius (max vertex radius) of a star-shaped mesh centred at 0."""
    V = V.astype(np.float64)
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    n = np.cross(b - a, c - a)
    # outward winding: every plane faces away from the centre
    assert np.all(np.einsum("ij,ij->i", n, a) > 0)
    r_in = np.min(np.einsum("ij,ij->i", n, a) / np.linalg.norm(n, axis=1))
    r_out = np.max(np.linalg.norm(V, axis=1))
    return r_in, r_out


def test_inside_parity_on_star_shaped_sphere():
    V, T = wl.noisy_sphere(24, 77, 0.3)
    V = V.astype(np.float32)
    r_in, r_out = star_regions(V, T)
    assert 0.3 < r_in < 1.0 < r_out < 1.5
    rng = np.random.default_rng(4)
    d = rng.normal(size=(4000, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    rad = np.concatenate([rng.uniform(0, 0.98 * r_in, 2000), rng.uniform(1.02 * r_out, 3.0, 2000)])
    P = (d * rad[:, None]).astype(np.float32)
    E = far_ends(V.astype(np.float64), P.astype(np.float64))
    ref = oracle.query(V, T, P, E)
    L = float(np.linalg.norm(V.max(0) - V.min(0)))
    deg = oracle.degenerate(V, T, P, E, 1e-6 * L)
    ok = deg == 0
    assert ok.mean() > 0.99
    expect_inside = np.arange(4000) < 2000
    assert np.array_equal((ref["count"][ok] & 1) == 1, expect_inside[ok])
    # a far end really lies outside the mesh box
    lo, hi = V.min(0), V.max(0)
    assert np.all(np.any((E < lo) | (E > hi), axis=1))


def test_inside_counts_open_surface_and_through_points():
    """On a closed cube every inside point has count 1, every outside point 0
    or 2 (the segment direction is generic, so no edge is hit)."""
    # unit cube [0,1]^3, 12 triangles, outward winding
    V = np.array([[x, y, z] for z in (0, 1) for y in (0, 1) for x in (0, 1)], np.float32)
    quads = [(0, 2, 3, 1), (4, 5, 7, 6), (0, 1, 5, 4), (2, 6, 7, 3), (0, 4, 6, 2), (1, 3, 7, 5)]
    T = np.array([t for a, b, c, d in quads for t in ((a, b, c), (a, c, d))], np.int32)
    rng = np.random.default_rng(9)
    P_in = rng.uniform(0.05, 0.95, (500, 3)).astype(np.float32)
    P_out = (rng.uniform(-1, 2, (3000, 3))).astype(np.float32)
    P_out = P_out[np.any((P_out < -0.05) | (P_out > 1.05), axis=1)][:500]
    P = np.concatenate([P_in, P_out])
    E = far_ends(V.astype(np.float64), P.astype(np.float64))
    ref = oracle.query(V, T, P, E)
    assert np.all(ref["count"][:500] == 1)
    assert np.all(ref["count"][500:] % 2 == 0)
