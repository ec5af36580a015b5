"""GPU build checks: Morton codes, the radix sort, and the tree validator.

The build follows the paper's Section 2 (triangle centroids, quantisation to
2^21 levels per axis inside the centroids' support interval, 64-bit Morton
codes, sort, binary radix tree) and Section 3.1 (bottom-up bounds with a
per-node arrival counter; the root kept as the left child of the last node
record).  The validator plays the role of the paper's tree-expansion debug
helpers (Section 3.1): every triangle appears in exactly one leaf, every
stored child box is exactly the union of the boxes below it, and the
reported height is the deepest internal level.
"""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _mesh(V, T, **kw):
    return rsi.Mesh(torch.from_numpy(V).cuda().contiguous(), torch.from_numpy(T).cuda().contiguous(), **kw)


def _spread(q):
    q = q.astype(np.uint64)
    out = np.zeros_like(q)
    for b in range(21):
        out |= ((q >> np.uint64(b)) & np.uint64(1)) << np.uint64(3 * b)
    return out


def _morton_reference(V, T):
    """Restatement of the quantisation and bit interleave in numpy float32."""
    a, b, c = V[T[:, 0]], V[T[:, 1]], V[T[:, 2]]
    cen = ((a + b) + c) * np.float32(1.0 / 3.0)
    lo = cen.min(0)
    hi = cen.max(0)
    ext = (hi - lo).astype(np.float32)
    q = np.zeros(cen.shape, np.uint64)
    for k in range(3):
        if ext[k] > 0:
            x = (cen[:, k] - lo[k]) / ext[k] * np.float32(2097152.0)
            x = np.minimum(np.maximum(x, np.float32(0)), np.float32(2097151.0))
            q[:, k] = x.astype(np.uint64)
    return (_spread(q[:, 0]) << np.uint64(2)) | (_spread(q[:, 1]) << np.uint64(1)) | _spread(q[:, 2])


def _validate(tree, V, T, leaf_size):
    n = tree["n_t"]
    boxes, refs, order = tree["boxes"], tree["refs"], tree["order"]
    tb_lo = np.minimum(np.minimum(V[T[:, 0]], V[T[:, 1]]), V[T[:, 2]])
    tb_hi = np.maximum(np.maximum(V[T[:, 0]], V[T[:, 1]]), V[T[:, 2]])
    seen = np.zeros(n, np.int32)
    max_depth = 0
    n_visited = 0

    def sub_box(ref, depth):
        nonlocal max_depth, n_visited
        if ref < 0:
            first = ref & 0x07FFFFFF
            cnt = ((ref >> 27) & 15) + 1
            assert cnt <= leaf_size
            ids = order[first:first + cnt]
            seen[first:first + cnt] += 1
            return tb_lo[ids].min(0), tb_hi[ids].max(0)
        n_visited += 1
        max_depth = max(max_depth, depth)
        lo_l, hi_l = sub_box(refs[ref, 0], depth + 1)
        lo_r, hi_r = sub_box(refs[ref, 1], depth + 1)
        assert np.array_equal(boxes[ref, 0:3], lo_l) and np.array_equal(boxes[ref, 3:6], hi_l)
        assert np.array_equal(boxes[ref, 6:9], lo_r) and np.array_equal(boxes[ref, 9:12], hi_r)
        return np.minimum(lo_l, lo_r), np.maximum(hi_l, hi_r)

    import sys
    sys.setrecursionlimit(10000)
    e = tree["entry"]
    lo, hi = sub_box(refs[e, 0], 1)
    assert np.array_equal(boxes[e, 0:3], lo) and np.array_equal(boxes[e, 3:6], hi)
    assert np.all(seen == 1), "every sorted position must sit in exactly one leaf"
    assert np.array_equal(np.sort(order), np.arange(n))
    assert tree["height"] == max_depth
    return n_visited


@pytest.mark.parametrize("leaf", [1, 2, 4, 16])
def test_tree_validator_heightfield(leaf):
    V, T = wl.config2_mesh()
    m = _mesh(V, T, leaf_size=leaf)
    tree = m.tree()
    keys = tree["keys"]
    assert np.all(keys[1:] >= keys[:-1])
    ref = _morton_reference(V, T)
    assert np.array_equal(keys, ref[tree["order"]])
    # stable: equal keys keep ascending triangle ids
    eq = keys[1:] == keys[:-1]
    assert np.all(tree["order"][1:][eq] > tree["order"][:-1][eq])
    _validate(tree, V, T, leaf)
    m.close()


def test_tree_validator_duplicates_and_tiny():
    # many identical centroids: duplicate Morton codes split by index
    V1, T1 = wl.sinusoid_heightfield(6, 1, 0.1)
    T = np.concatenate([T1] * 40, 0)
    m = _mesh(V1, T)
    tree = m.tree()
    _validate(tree, V1, T, 1)
    m.close()
    for n in (1, 2, 3):
        V = np.random.default_rng(n).uniform(size=(3 * n, 3)).astype(np.float32)
        Tn = np.arange(3 * n, dtype=np.int32).reshape(n, 3)
        m = _mesh(V, Tn)
        _validate(m.tree(), V, Tn, 1)
        m.close()


def test_sort_large_mesh():
    V, T = wl.noisy_sphere(60, 12, 0.3)  # 72,000 triangles: several sort tiles
    m = _mesh(V, T)
    tree = m.tree()
    assert np.array_equal(tree["keys"], np.sort(_morton_reference(V, T), kind="stable"))
    assert np.array_equal(tree["order"], np.argsort(_morton_reference(V, T), kind="stable"))
    _validate(tree, V, T, 1)
    m.close()


@pytest.mark.parametrize("n_cluster", [300, 2500, 9000])
def test_sort_clustered_buckets(n_cluster):
    """Most triangles in one corner cell of the mesh box and a few far away:
    the small-sort path groups the keys by their top 8 bits and then sorts
    each group, in LDS up to 2048 elements and over device memory above
    that; the sorted keys and the stable order must match numpy's."""
    rng = np.random.default_rng(n_cluster)
    c = rng.uniform(0.0, 1e-3, size=(n_cluster, 1, 3)) + rng.uniform(-1e-5, 1e-5, size=(n_cluster, 3, 3))
    far = rng.uniform(0.5, 1.0, size=(40, 1, 3)) + rng.uniform(-1e-2, 1e-2, size=(40, 3, 3))
    tris = np.concatenate([c, far], 0).astype(np.float32)
    V = tris.reshape(-1, 3)
    T = np.arange(V.shape[0], dtype=np.int32).reshape(-1, 3)
    m = _mesh(V, T)
    tree = m.tree()
    ref = _morton_reference(V, T)
    assert np.array_equal(tree["keys"], np.sort(ref, kind="stable"))
    assert np.array_equal(tree["order"], np.argsort(ref, kind="stable"))
    _validate(tree, V, T, 1)
    m.close()


@pytest.mark.parametrize("kind", ["sphere", "clustered"])
def test_sort_large_inputs(kind):
    """Above 131,072 keys the bucket sort runs on a scanned histogram table:
    a sphere of 180,500 triangles spreads over many buckets, each sorted in
    LDS; a mesh with most triangles in one corner cell puts them in one
    bucket, which streams through device memory.  Either way the keys and
    the stable order must match numpy's."""
    if kind == "sphere":
        V, T = wl.noisy_sphere(95, 12, 0.3)
    else:
        rng = np.random.default_rng(7)
        c = rng.uniform(0.0, 1e-3, size=(140_000, 1, 3)) + rng.uniform(-1e-5, 1e-5, size=(140_000, 3, 3))
        far = rng.uniform(0.5, 1.0, size=(200, 1, 3)) + rng.uniform(-1e-2, 1e-2, size=(200, 3, 3))
        V = np.concatenate([c, far], 0).astype(np.float32).reshape(-1, 3)
        T = np.arange(V.shape[0], dtype=np.int32).reshape(-1, 3)
    assert T.shape[0] > 131_072
    m = _mesh(V, T)
    tree = m.tree()
    ref = _morton_reference(V, T)
    assert np.array_equal(tree["keys"], np.sort(ref, kind="stable"))
    assert np.array_equal(tree["order"], np.argsort(ref, kind="stable"))
    _validate(tree, V, T, 1)
    m.close()
