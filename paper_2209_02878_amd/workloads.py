"""Seeded synthetic workloads: triangle meshes and line segments.

This module only draws inputs.  It holds none of the intersection arithmetic,
so both the FP64 oracle and the GPU path can be fed from it without sharing
any of the method's code.

The paper measures on an unpublished 29,284-triangle terrain-like surface and
10M random rays (Section 2, Table 1 and Section 4.1); those inputs are not
available, so the heightfields and noisy spheres generated here stand in for
them, with the sizes of the paper's workload.

Every generator returns numpy arrays in the layouts of the paper's input files
(Section 2.5): vertices float32 [N_v, 3], triangles int32 [N_t, 3], segment
starts and ends float32 [N_r, 3].
"""
from __future__ import annotations

import math
from dataclasses import dataclass

import numpy as np

BASE_SEED = 20902878


def seed_for(config: int, stream: int) -> int:
    """Seed of `stream` (1 = mesh, 2 = segments, 3 = check subset, 4 = target)
    for workload `config` (1-based)."""
    return BASE_SEED + 10 * config + stream


# ---------------------------------------------------------------- noise ----

def _fade(t):
    # quintic smoothstep 6t^5 - 15t^4 + 10t^3
    return t * t * t * (t * (t * 6.0 - 15.0) + 10.0)


def value_noise_2d(rng: np.random.Generator, x, y, octaves: int, base_freq: int):
    """Sum over octaves o of 2^-o * lattice value noise at frequency base*2^o.

    Lattice values are U[-1, 1] on an (f+1) x (f+1) grid over [0, 1]^2 and are
    blended with the quintic fade.  x, y are float64 arrays in [0, 1].
    """
    x = np.asarray(x, np.float64)
    y = np.asarray(y, np.float64)
    out = np.zeros(np.broadcast(x, y).shape, np.float64)
    for o in range(octaves):
        f = base_freq * (2 ** o)
        lat = rng.uniform(-1.0, 1.0, size=(f + 1, f + 1))
        X = np.clip(x, 0.0, 1.0) * f
        Y = np.clip(y, 0.0, 1.0) * f
        i = np.minimum(np.floor(X).astype(np.int64), f - 1)
        j = np.minimum(np.floor(Y).astype(np.int64), f - 1)
        fx = _fade(X - i)
        fy = _fade(Y - j)
        a = lat[i, j] * (1 - fx) + lat[i + 1, j] * fx
        b = lat[i, j + 1] * (1 - fx) + lat[i + 1, j + 1] * fx
        out += (2.0 ** -o) * (a * (1 - fy) + b * fy)
    return out


def value_noise_3d(rng: np.random.Generator, p, octaves: int, base_freq: int):
    """3D lattice value noise over [-1, 1]^3 (points p float64 [n, 3])."""
    q = (np.clip(np.asarray(p, np.float64), -1.0, 1.0) + 1.0) * 0.5
    out = np.zeros(q.shape[0], np.float64)
    for o in range(octaves):
        f = base_freq * (2 ** o)
        lat = rng.uniform(-1.0, 1.0, size=(f + 1, f + 1, f + 1))
        X = q * f
        idx = np.minimum(np.floor(X).astype(np.int64), f - 1)
        w = _fade(X - idx)
        acc = np.zeros(q.shape[0], np.float64)
        for dx in (0, 1):
            wx = w[:, 0] if dx else 1 - w[:, 0]
            for dy in (0, 1):
                wy = w[:, 1] if dy else 1 - w[:, 1]
                for dz in (0, 1):
                    wz = w[:, 2] if dz else 1 - w[:, 2]
                    acc += wx * wy * wz * lat[idx[:, 0] + dx, idx[:, 1] + dy, idx[:, 2] + dz]
        out += (2.0 ** -o) * acc
    return out


# --------------------------------------------------------------- meshes ----

def grid_triangles(n: int) -> np.ndarray:
    """Triangles of an n x n vertex grid; vertex (i, j) has index j*n + i.

    Each cell is split along its (i, j)-(i+1, j+1) diagonal; both triangles
    are counter-clockwise seen from +z.  Triangle 2*(j*(n-1)+i) is the lower
    right one, 2*(j*(n-1)+i)+1 the upper left one.
    """
    i, j = np.meshgrid(np.arange(n - 1), np.arange(n - 1), indexing="xy")
    i = i.ravel()
    j = j.ravel()
    v00 = j * n + i
    v10 = v00 + 1
    v01 = v00 + n
    v11 = v01 + 1
    tris = np.empty((2 * (n - 1) * (n - 1), 3), np.int64)
    tris[0::2] = np.stack([v00, v10, v11], 1)
    tris[1::2] = np.stack([v00, v11, v01], 1)
    return tris.astype(np.int32)


def grid_xy(n: int):
    g = np.arange(n, dtype=np.float64) / (n - 1)
    x, y = np.meshgrid(g, g, indexing="xy")
    return x.ravel(), y.ravel()


def sinusoid_heightfield(n: int, seed: int, amplitude: float = 0.1):
    """Heightfield whose z is a sum of 4 seeded plane waves scaled to max|z| = amplitude."""
    rng = np.random.default_rng(seed)
    x, y = grid_xy(n)
    z = np.zeros_like(x)
    for _ in range(4):
        fx, fy = rng.integers(1, 4, size=2)
        phi = rng.uniform(0.0, 2.0 * math.pi)
        z += np.sin(2.0 * math.pi * (fx * x + fy * y) + phi)
    z *= amplitude / np.max(np.abs(z))
    V = np.stack([x, y, z], 1).astype(np.float32)
    return V, grid_triangles(n)


def noise_heightfield(n: int, seed: int, amplitude: float = 0.2, jitter: float = 0.0,
                      octaves: int = 6, base_freq: int = 4):
    """Heightfield whose z is seeded value noise scaled to max|z| = amplitude,
    with optional uniform xy jitter of +-jitter."""
    rng = np.random.default_rng(seed)
    x, y = grid_xy(n)
    z = value_noise_2d(rng, x, y, octaves, base_freq)
    z *= amplitude / np.max(np.abs(z))
    if jitter > 0:
        x = x + rng.uniform(-jitter, jitter, size=x.shape)
        y = y + rng.uniform(-jitter, jitter, size=y.shape)
    V = np.stack([x, y, z], 1).astype(np.float32)
    return V, grid_triangles(n)


_ICO_V = None


def _icosahedron():
    p = (1.0 + 5.0 ** 0.5) / 2.0
    v = np.array([[-1, p, 0], [1, p, 0], [-1, -p, 0], [1, -p, 0],
                  [0, -1, p], [0, 1, p], [0, -1, -p], [0, 1, -p],
                  [p, 0, -1], [p, 0, 1], [-p, 0, -1], [-p, 0, 1]], np.float64)
    v /= np.linalg.norm(v, axis=1, keepdims=True)
    f = np.array([[0, 11, 5], [0, 5, 1], [0, 1, 7], [0, 7, 10], [0, 10, 11],
                  [1, 5, 9], [5, 11, 4], [11, 10, 2], [10, 7, 6], [7, 1, 8],
                  [3, 9, 4], [3, 4, 2], [3, 2, 6], [3, 6, 8], [3, 8, 9],
                  [4, 9, 5], [2, 4, 11], [6, 2, 10], [8, 6, 7], [9, 8, 1]], np.int64)
    return v, f


def geodesic_sphere(freq: int):
    """Unit geodesic sphere of frequency `freq`: every icosahedron face is split
    into freq^2 triangles and the vertices are projected onto the sphere.

    Returns float64 unit vertices [10 f^2 + 2, 3] and int32 triangles
    [20 f^2, 3], outward (counter-clockwise seen from outside) winding.
    """
    iv, faces = _icosahedron()
    f = freq
    # integer barycentric lattice on one face: (a, b) with a + b <= f
    ab = [(a, b) for a in range(f + 1) for b in range(f + 1 - a)]
    ab = np.array(ab, np.int64)
    loc = {(int(a), int(b)): k for k, (a, b) in enumerate(ab)}
    small = []
    for a in range(f):
        for b in range(f - a):
            small.append((loc[(a, b)], loc[(a + 1, b)], loc[(a, b + 1)]))
            if a + b < f - 1:
                small.append((loc[(a + 1, b)], loc[(a + 1, b + 1)], loc[(a, b + 1)]))
    small = np.array(small, np.int64)
    # a global key for each lattice point: identical points on shared edges
    # and corners get identical integer keys (weights over icosahedron vertices)
    keys = {}
    verts = []
    tri_out = np.empty((20 * small.shape[0], 3), np.int64)
    for fi, (A, B, C) in enumerate(faces):
        ids = np.empty(ab.shape[0], np.int64)
        for k, (a, b) in enumerate(ab):
            c = f - a - b
            w = {}
            for vid, wt in ((A, c), (B, a), (C, b)):
                if wt:
                    w[int(vid)] = w.get(int(vid), 0) + int(wt)
            key = tuple(sorted(w.items()))
            g = keys.get(key)
            if g is None:
                g = len(verts)
                keys[key] = g
                pt = sum(iv[vid] * wt for vid, wt in key) / f
                verts.append(pt)
            ids[k] = g
        tri_out[fi * small.shape[0]:(fi + 1) * small.shape[0]] = ids[small]
    V = np.array(verts, np.float64)
    V /= np.linalg.norm(V, axis=1, keepdims=True)
    # make every triangle wind outward
    a, b, c = V[tri_out[:, 0]], V[tri_out[:, 1]], V[tri_out[:, 2]]
    n = np.cross(b - a, c - a)
    flip = np.einsum("ij,ij->i", n, a + b + c) < 0
    tri_out[flip] = tri_out[flip][:, [0, 2, 1]]
    return V, tri_out.astype(np.int32)


def noisy_sphere(freq: int, seed: int, amplitude: float = 0.3, octaves: int = 4,
                 base_freq: int = 2):
    """Closed star-shaped surface: a geodesic sphere whose radius is
    1 + amplitude * N(p) / max|N| with N seeded 3D value noise at the unit
    direction p."""
    rng = np.random.default_rng(seed)
    U, T = geodesic_sphere(freq)
    nz = value_noise_3d(rng, U, octaves, base_freq)
    r = 1.0 + amplitude * nz / np.max(np.abs(nz))
    V = (U * r[:, None]).astype(np.float32)
    return V, T


# ------------------------------------------------------------- segments ----

def segments_in_box(rng, lo, hi, n, scale: float = 1.0):
    """Both ends uniform in the box [lo, hi] scaled by `scale` about its centre."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    c = 0.5 * (lo + hi)
    h = 0.5 * (hi - lo) * scale
    S = rng.uniform(c - h, c + h, size=(n, 3))
    E = rng.uniform(c - h, c + h, size=(n, 3))
    return S.astype(np.float32), E.astype(np.float32)


def segments_random_dir(rng, lo, hi, n, len_lo=0.01, len_hi=1.0):
    """Start uniform in the box, direction uniform on the sphere, length
    log-uniform over [len_lo, len_hi]."""
    lo = np.asarray(lo, np.float64)
    hi = np.asarray(hi, np.float64)
    S = rng.uniform(lo, hi, size=(n, 3))
    d = rng.standard_normal(size=(n, 3))
    d /= np.linalg.norm(d, axis=1, keepdims=True)
    ln = np.exp(rng.uniform(math.log(len_lo), math.log(len_hi), size=(n, 1)))
    E = S + ln * d
    return S.astype(np.float32), E.astype(np.float32)


def segments_near_vertical(rng, n, lo=0.02, hi=0.98, dxy=0.01, z0=1.0, z1=-1.0):
    xy = rng.uniform(lo, hi, size=(n, 2))
    dd = rng.uniform(-dxy, dxy, size=(n, 2))
    S = np.concatenate([xy, np.full((n, 1), z0)], 1)
    E = np.concatenate([xy + dd, np.full((n, 1), z1)], 1)
    return S.astype(np.float32), E.astype(np.float32)


# ------------------------------------------------------------- configs -----

@dataclass
class Workload:
    name: str
    V: np.ndarray
    T: np.ndarray
    S: np.ndarray
    E: np.ndarray
    capacity_k: int = 0
    note: str = ""

    @property
    def n_v(self):
        return self.V.shape[0]

    @property
    def n_t(self):
        return self.T.shape[0]

    @property
    def n_r(self):
        return self.S.shape[0]


def mesh_bbox(V):
    V = np.asarray(V, np.float64)
    return V.min(0), V.max(0)


def config1(n_r: int = 100_000) -> Workload:
    """Sinusoid heightfield on a 32 x 32 grid (1,922 triangles), 100k segments
    with both ends uniform in [0,1]^2 x [-0.3, 0.3]; boolean output."""
    V, T = sinusoid_heightfield(32, seed_for(1, 1), 0.1)
    rng = np.random.default_rng(seed_for(1, 2))
    S, E = segments_in_box(rng, [0, 0, -0.3], [1, 1, 0.3], n_r)
    return Workload("heightfield-1922tri-bool-100k", V, T, S, E)


def config2_mesh():
    return noise_heightfield(123, seed_for(2, 1), 0.2, jitter=1e-3)


def config2(n_r: int = 10_000_000, mesh=None) -> Workload:
    """Value-noise heightfield on a 123 x 123 grid (29,768 triangles) with
    1e-3 xy jitter; segments start uniform in the mesh box, point uniformly on
    the sphere and have log-uniform length in [0.01, 1]."""
    V, T = mesh if mesh is not None else config2_mesh()
    lo, hi = mesh_bbox(V)
    rng = np.random.default_rng(seed_for(2, 2))
    S, E = segments_random_dir(rng, lo, hi, n_r)
    return Workload("heightfield-29768tri-10Mseg", V, T, S, E, capacity_k=4)


def config3_mesh(freq: int = 158):
    return noisy_sphere(freq, seed_for(3, 1), 0.3)


def config3(n_r: int = 10_000_000, freq: int = 158, mesh=None) -> Workload:
    """Noisy closed sphere (frequency-158 geodesic, 499,280 triangles, +-30%
    radius noise); both segment ends uniform in 1.5x the mesh box; all-hits
    with capacity 4 plus first hit."""
    V, T = mesh if mesh is not None else config3_mesh(freq)
    lo, hi = mesh_bbox(V)
    rng = np.random.default_rng(seed_for(3, 2))
    S, E = segments_in_box(rng, lo, hi, n_r, scale=1.5)
    return Workload(f"noisysphere-{T.shape[0]}tri-{n_r}seg", V, T, S, E, capacity_k=4)


def config4_mesh(n: int = 317):
    return noise_heightfield(n, seed_for(4, 1), 0.2, jitter=0.0)


def config4_target(n: int = 317):
    """Second seeded noise surface g on the same grid (target heights)."""
    return noise_heightfield(n, seed_for(4, 4), 0.2, jitter=0.0)


def config4(n_r: int = 4_000_000, n: int = 317) -> Workload:
    """Differentiable first hit: 317 x 317 heightfield (199,712 triangles),
    4M near-vertical segments from z = 1 to z = -1."""
    V, T = config4_mesh(n)
    rng = np.random.default_rng(seed_for(4, 2))
    S, E = segments_near_vertical(rng, n_r)
    return Workload(f"heightfield-{T.shape[0]}tri-{n_r}seg-diff", V, T, S, E)


def inside_points(V, n: int, seed: int) -> np.ndarray:
    """Points for the odd-parity inside test: uniform in 1.5x the mesh box
    (about centre), FP32."""
    lo, hi = mesh_bbox(V)
    c, h = 0.5 * (lo + hi), 0.75 * (hi - lo)
    rng = np.random.default_rng(seed)
    return rng.uniform(c - h, c + h, (n, 3)).astype(np.float32)


def subset(n_total: int, n_pick: int, seed: int) -> np.ndarray:
    """Seeded sorted sample of segment indices."""
    if n_pick >= n_total:
        return np.arange(n_total, dtype=np.int64)
    rng = np.random.default_rng(seed)
    return np.sort(rng.choice(n_total, size=n_pick, replace=False)).astype(np.int64)


def config5(n_meshes: int = 64, tri_lo: float = 1e3, tri_hi: float = 2e5, seg_lo: float = 1e4,
            seg_hi: float = 2e6, seed: int | None = None):
    """Batched workload: meshes that are heightfields (value noise, grid
    n = round(sqrt(N_t / 2)) + 1) or noisy geodesic spheres (frequency
    round(sqrt(N_t / 20))) with equal probability, target triangle counts
    log-uniform in [tri_lo, tri_hi]; per mesh a log-uniform number of
    segments in [seg_lo, seg_hi], drawn like the 29,768-triangle workload's
    (heightfields) or the closed sphere's (spheres).  Returns a list of
    Workload objects."""
    rng = np.random.default_rng(seed_for(5, 1) if seed is None else seed)
    out = []
    for m in range(n_meshes):
        target = math.exp(rng.uniform(math.log(tri_lo), math.log(tri_hi)))
        n_seg = int(math.exp(rng.uniform(math.log(seg_lo), math.log(seg_hi))))
        mseed = int(rng.integers(1 << 31))
        srng = np.random.default_rng(int(rng.integers(1 << 31)))
        if rng.uniform() < 0.5:
            n = max(2, int(round(math.sqrt(target / 2.0))) + 1)
            V, T = noise_heightfield(n, mseed, 0.2, jitter=0.25 / (n - 1))
            lo, hi = mesh_bbox(V)
            S, E = segments_random_dir(srng, lo, hi, n_seg)
            kind = "heightfield"
        else:
            f = max(1, int(round(math.sqrt(target / 20.0))))
            V, T = noisy_sphere(f, mseed, 0.3)
            lo, hi = mesh_bbox(V)
            S, E = segments_in_box(srng, lo, hi, n_seg, scale=1.5)
            kind = "sphere"
        out.append(Workload(f"{kind}-{T.shape[0]}tri-{n_seg}seg", V, T, S, E))
    return out
