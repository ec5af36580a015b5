"""The box test of the traversal never rejects a box that the segment touches.

The query kernel culls with a slab test in FP32: per axis the parameters
(plane - o) * (1/d), each a subtraction and a product, with direction
components below the smallest normal FP32 value (2^-126) in magnitude
replaced by +-2^-126, the reciprocal
taken by the hardware instruction (within 1 ulp), and acceptance when
near <= far * (1 + 2^-20).  This test restates that arithmetic in Python
(FP32 operations through numpy; the reciprocal correctly rounded and then
moved by -1, 0 or +1 ulp at random, covering any result the instruction may
give) and checks it against an
exact rational slab test on the same FP32 segment, over random and
adversarial cases: endpoints on faces, nearly parallel segments, flat boxes,
origins far from short segments, zero and tiny direction components.  A
touched box must always be accepted; the only exception is a segment with an
exactly zero direction component lying in a box face plane, which can meet
the triangles inside only on their boundary.
"""
from fractions import Fraction

import numpy as np
import pytest

F32 = np.float32


_ulp_rng = np.random.default_rng(5)


def slab_accepts(s, e, lo, hi, tmax=F32(1.0)):
    d = (e - s).astype(F32)
    tiny = F32(2.0 ** -126)
    g = np.where(np.abs(d) < tiny, np.copysign(tiny, d), d).astype(F32)
    inv = (F32(1.0) / g).astype(F32)
    for k in range(3):
        step = _ulp_rng.integers(-1, 2)
        if step:
            inv[k] = np.nextafter(inv[k], F32(np.inf) if step > 0 else F32(-np.inf)).astype(F32)
    t0 = ((lo - s).astype(F32) * inv).astype(F32)
    t1 = ((hi - s).astype(F32) * inv).astype(F32)
    near = max(max(min(t0[0], t1[0]), min(t0[1], t1[1])), max(min(t0[2], t1[2]), F32(0.0)))
    far = min(min(max(t0[0], t1[0]), max(t0[1], t1[1])), min(max(t0[2], t1[2]), tmax))
    return bool(near <= F32(far * F32(1.0 + 2.0 ** -20)))


def exact_touch(s, e, lo, hi, tmax=1.0):
    """Does o + t d (d the FP32 difference e - s, as the kernel uses it),
    t in [0, tmax], meet the closed box?  Also reports whether the only
    contact is the zero-direction-in-face-plane exception."""
    d = (e - s).astype(F32)
    a, b = Fraction(0), Fraction(float(tmax))
    face_plane = False
    for k in range(3):
        o, dk = Fraction(float(s[k])), Fraction(float(d[k]))
        l, h = Fraction(float(lo[k])), Fraction(float(hi[k]))
        if dk == 0:
            if o < l or o > h:
                return False, False
            if o == l or o == h:
                face_plane = True
            continue
        u, v = (l - o) / dk, (h - o) / dk
        a, b = max(a, min(u, v)), min(b, max(u, v))
    return a <= b, face_plane


def _check(cases):
    touched = accepted_extra = 0
    for s, e, lo, hi in cases:
        ok, face = exact_touch(s, e, lo, hi)
        acc = slab_accepts(s, e, lo, hi)
        if ok:
            touched += 1
            if not face:
                assert acc, (s, e, lo, hi)
        elif acc:
            accepted_extra += 1
    return touched, accepted_extra


def _box(rng, c, size):
    a = (c + rng.uniform(-size, size, 3)).astype(F32)
    b = (c + rng.uniform(-size, size, 3)).astype(F32)
    return np.minimum(a, b), np.maximum(a, b)


def test_random_segments_and_boxes():
    rng = np.random.default_rng(20902878)
    cases = []
    for _ in range(3000):
        c = rng.uniform(-1, 1, 3)
        lo, hi = _box(rng, c, rng.uniform(1e-3, 0.5))
        s = (c + rng.uniform(-0.6, 0.6, 3)).astype(F32)
        e = (s + rng.normal(size=3) * rng.uniform(0.01, 2.0)).astype(F32)
        cases.append((s, e, lo, hi))
    touched, _ = _check(cases)
    assert touched > 30


def test_endpoints_and_crossings_on_faces():
    rng = np.random.default_rng(7)
    cases = []
    for _ in range(2000):
        lo, hi = _box(rng, rng.uniform(-1, 1, 3), rng.uniform(1e-3, 0.3))
        # a point on a face of the box (exact FP32 coordinates) as start or end
        p = rng.uniform(lo, hi).astype(F32)
        k = rng.integers(3)
        p[k] = lo[k] if rng.uniform() < 0.5 else hi[k]
        q = (p + rng.normal(size=3) * rng.uniform(1e-4, 1.0)).astype(F32)
        cases.append((p, q, lo, hi) if rng.uniform() < 0.5 else (q, p, lo, hi))
    touched, _ = _check(cases)
    assert touched > 500


def test_nearly_parallel_and_tiny_components():
    rng = np.random.default_rng(11)
    cases = []
    for _ in range(2000):
        lo, hi = _box(rng, rng.uniform(-1, 1, 3), rng.uniform(1e-3, 0.3))
        s = rng.uniform(lo - 0.2, hi + 0.2).astype(F32)
        dvec = rng.normal(size=3)
        k = rng.integers(3)
        dvec[k] *= 10.0 ** rng.uniform(-30, -3) if rng.uniform() < 0.8 else 0.0
        e = (s.astype(np.float64) + dvec * rng.uniform(0.05, 1.0)).astype(F32)
        # the start on the face plane of the tiny axis half of the time
        if rng.uniform() < 0.5:
            s[k] = lo[k]
            e[k] = F32(np.float64(lo[k]) + dvec[k])
        cases.append((s, e, lo, hi))
    touched, _ = _check(cases)
    assert touched > 100


def test_flat_boxes_and_far_origins():
    rng = np.random.default_rng(13)
    cases = []
    for _ in range(2000):
        c = rng.uniform(-1, 1, 3) * (1000.0 if rng.uniform() < 0.3 else 1.0)
        lo, hi = _box(rng, c, rng.uniform(1e-4, 0.2))
        k = rng.integers(3)
        hi[k] = lo[k]  # flat in one axis, like an axis-aligned triangle's box
        # short segments through a point of the box
        p = rng.uniform(lo, hi)
        dvec = rng.normal(size=3) * rng.uniform(1e-3, 0.5)
        a = rng.uniform(0, 1)
        s = (p - a * dvec).astype(F32)
        e = (p + (1 - a) * dvec).astype(F32)
        cases.append((s, e, lo, hi))
    touched, _ = _check(cases)
    assert touched > 500


@pytest.mark.parametrize("scale", [1e-34, 1e-30, 1.0, 1e6])
def test_axis_parallel_segments_at_any_scale(scale):
    """Zero direction components: exact unless the segment lies in a face plane."""
    rng = np.random.default_rng(17)
    cases = []
    for _ in range(500):
        lo, hi = _box(rng, rng.uniform(-1, 1, 3), rng.uniform(1e-3, 0.3))
        lo, hi = (lo * scale).astype(F32), (hi * scale).astype(F32)
        s = (rng.uniform(-1.2, 1.2, 3) * scale).astype(F32)
        e = s.copy()
        k = rng.integers(3)
        e[k] = F32(s[k] + scale * rng.uniform(-2, 2))
        cases.append((s, e, lo, hi))
    _check(cases)
