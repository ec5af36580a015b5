"""Thin ctypes binding of librsi.so (include/rsi.h).

Argument marshalling only: every step of the build and the queries runs in
the library's HIP kernels.  torch supplies device memory and the stream.  If
librsi.so has not been built, every call raises RuntimeError; there is no
fallback path.

Low-level functions carry the C names (rsi_build, rsi_query, ...).  `Mesh`
wraps a handle and allocates output tensors.
"""
from __future__ import annotations

import ctypes
import os

import torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "librsi.so")

RSI_OK, RSI_E_INVALID, RSI_E_NOMEM, RSI_E_HIP, RSI_E_OVERFLOW = range(5)
RSI_BOOL, RSI_FIRST_HIT, RSI_ALL_HITS, RSI_COUNT = 1, 2, 4, 8
MODE_NAMES = {"bool": RSI_BOOL, "first": RSI_FIRST_HIT, "all": RSI_ALL_HITS, "count": RSI_COUNT}

EXPORTED = [
    "rsi_build", "rsi_rebuild", "rsi_refit", "rsi_query", "rsi_query_noalloc", "rsi_compact", "rsi_segment_order", "rsi_gather_segments", "rsi_inside", "rsi_first_hit_backward",
    "rsi_spill_info", "rsi_spill_read", "rsi_query_stats",
    "rsi_set_counting", "rsi_get_counters", "rsi_get_tree_info", "rsi_get_mesh_info", "rsi_export_tree",
    "rsi_batch_create", "rsi_batch_rebuild", "rsi_batch_query", "rsi_batch_capture", "rsi_batch_replay",
    "rsi_set_opts", "rsi_get_opts", "rsi_tune",
    "rsi_destroy", "rsi_status_str", "rsi_last_error",
]


class RsiError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"{msg} (status {status})")
        self.status = status


class rsi_opts(ctypes.Structure):
    _fields_ = [("leaf_size", ctypes.c_int32), ("block_size", ctypes.c_int32),
                ("defer_lanes", ctypes.c_int32), ("refill_lanes", ctypes.c_int32),
                ("chunk", ctypes.c_int32), ("stack_depth", ctypes.c_int32), ("branching", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


class rsi_tune_job(ctypes.Structure):
    _fields_ = [("V", ctypes.c_void_p), ("n_v", ctypes.c_int64), ("T", ctypes.c_void_p), ("S", ctypes.c_void_p),
                ("E", ctypes.c_void_p), ("n_r", ctypes.c_int64), ("out", ctypes.c_void_p), ("bS", ctypes.c_void_p),
                ("bE", ctypes.c_void_p), ("b_nr", ctypes.c_void_p), ("b_outs", ctypes.c_void_p),
                ("mode", ctypes.c_uint32), ("reserved", ctypes.c_int32)]


class rsi_outputs(ctypes.Structure):
    _fields_ = [("hit", ctypes.c_void_p), ("tri", ctypes.c_void_p), ("t", ctypes.c_void_p),
                ("uv", ctypes.c_void_p), ("point", ctypes.c_void_p), ("count", ctypes.c_void_p),
                ("ids", ctypes.c_void_p), ("ts", ctypes.c_void_p), ("capacity", ctypes.c_int32),
                ("reserved", ctypes.c_int32), ("spill_off", ctypes.c_void_p), ("spill_ids", ctypes.c_void_p),
                ("spill_ts", ctypes.c_void_p), ("spill_cap", ctypes.c_int64)]


class rsi_stats(ctypes.Structure):
    _fields_ = [("bad_index", ctypes.c_int32), ("build_inconsistent", ctypes.c_int32),
                ("walk_cut", ctypes.c_int32), ("stack_dropped", ctypes.c_int32),
                ("overflow_full", ctypes.c_int32), ("reserved", ctypes.c_int32),
                ("deep_segments", ctypes.c_int64), ("overflow_segments", ctypes.c_int64),
                ("overflow_crossings", ctypes.c_int64), ("arena_records", ctypes.c_int64),
                ("pool_capacity", ctypes.c_int64)]


class rsi_counters(ctypes.Structure):
    _fields_ = [("node_visits", ctypes.c_uint64), ("box_tests", ctypes.c_uint64),
                ("tri_tests", ctypes.c_uint64), ("segments", ctypes.c_uint64),
                ("wave_loops", ctypes.c_uint64), ("wave_node_steps", ctypes.c_uint64),
                ("wave_leaf_phases", ctypes.c_uint64), ("wave_refills", ctypes.c_uint64),
                ("lanes_blocked", ctypes.c_uint64), ("lanes_waiting", ctypes.c_uint64),
                ("wave_leaf_rounds", ctypes.c_uint64), ("leaf_lanes", ctypes.c_uint64)]


class rsi_tree_info(ctypes.Structure):
    _fields_ = [("n_t", ctypes.c_int64), ("n_nodes", ctypes.c_int64), ("height", ctypes.c_int32),
                ("leaf_size", ctypes.c_int32), ("entry", ctypes.c_int32), ("n_meshes", ctypes.c_int32)]


_lib = None


def lib():
    """Load librsi.so (raises RuntimeError when it is missing)."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built: run __graft_entry__.build() "
                           "(hipcc --offload-arch=gfx950); there is no fallback path")
    L = ctypes.CDLL(LIB_PATH)
    P, i64, i32, u32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32, ctypes.c_uint32
    H = ctypes.c_void_p
    L.rsi_build.argtypes = [P, i64, P, i64, ctypes.POINTER(rsi_opts), P, ctypes.POINTER(H)]
    L.rsi_rebuild.argtypes = [H, P, i64, P, P]
    L.rsi_refit.argtypes = [H, P, i64, P]
    L.rsi_query.argtypes = [H, P, P, i64, u32, ctypes.POINTER(rsi_outputs), P]
    L.rsi_query_noalloc.argtypes = [H, P, P, i64, u32, ctypes.POINTER(rsi_outputs), P]
    L.rsi_inside.argtypes = [H, P, i64, P, P, P, P]
    L.rsi_segment_order.argtypes = [H, P, P, i64, P, P]
    L.rsi_gather_segments.argtypes = [H, P, P, P, i64, P, P, P]
    L.rsi_compact.argtypes = [H, P, P, P, P, P, P, i64, P, P, P, P, ctypes.POINTER(i64), P]
    L.rsi_first_hit_backward.argtypes = [H, P, i64, P, P, i64, P, P, P, P, P, P, P, P]
    L.rsi_spill_info.argtypes = [H, ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.rsi_spill_read.argtypes = [H, P, P, P, P, P, P]
    L.rsi_query_stats.argtypes = [H, ctypes.POINTER(rsi_stats)]
    L.rsi_set_counting.argtypes = [H, ctypes.c_int]
    L.rsi_get_counters.argtypes = [H, ctypes.POINTER(rsi_counters)]
    L.rsi_get_tree_info.argtypes = [H, ctypes.POINTER(rsi_tree_info)]
    L.rsi_export_tree.argtypes = [H, P, P, P, P]
    L.rsi_get_mesh_info.argtypes = [H, i32, ctypes.POINTER(i64), ctypes.POINTER(i64), ctypes.POINTER(i32)]
    L.rsi_batch_create.argtypes = [i32, P, P, P, P, ctypes.POINTER(rsi_opts), P, ctypes.POINTER(H)]
    L.rsi_batch_rebuild.argtypes = [H, P]
    L.rsi_batch_query.argtypes = [H, P, P, P, u32, P, P]
    L.rsi_batch_capture.argtypes = [H, P, P, P, u32, P, ctypes.c_int, P]
    L.rsi_batch_replay.argtypes = [H, P]
    L.rsi_set_opts.argtypes = [H, ctypes.POINTER(rsi_opts)]
    L.rsi_get_opts.argtypes = [H, ctypes.POINTER(rsi_opts)]
    L.rsi_tune.argtypes = [H, ctypes.POINTER(rsi_tune_job), P, i32, i32, P, ctypes.POINTER(i32), P]
    L.rsi_destroy.argtypes = [H]
    L.rsi_destroy.restype = None
    L.rsi_status_str.argtypes = [ctypes.c_int]
    L.rsi_status_str.restype = ctypes.c_char_p
    L.rsi_last_error.argtypes = []
    L.rsi_last_error.restype = ctypes.c_char_p
    for name in EXPORTED:
        if name not in ("rsi_destroy", "rsi_status_str", "rsi_last_error"):
            getattr(L, name).restype = ctypes.c_int
    _lib = L
    return L


def _check(status):
    if status != RSI_OK:
        L = lib()
        raise RsiError(status, (L.rsi_last_error() or b"").decode() or L.rsi_status_str(status).decode())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _dev_f32(x, name, cols=3):
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.float32 or not x.is_contiguous() or x.dim() != 2 or x.shape[1] != cols:
        raise TypeError(f"{name} must be a contiguous float32 [n, {cols}] tensor")
    return x


def _dev_i32(x, name):
    if not (isinstance(x, torch.Tensor) and x.is_cuda):
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if x.dtype != torch.int32 or not x.is_contiguous() or x.dim() != 2 or x.shape[1] != 3:
        raise TypeError(f"{name} must be a contiguous int32 [n, 3] tensor")
    return x


# ------------------------------------------------------------ C functions --

def rsi_build(V, T, leaf_size=0, block_size=0, stream=None, defer_lanes=0, refill_lanes=0, chunk=0,
              stack_depth=0, branching=0):
    V = _dev_f32(V, "V")
    T = _dev_i32(T, "T")
    h = ctypes.c_void_p()
    o = rsi_opts(leaf_size, block_size, defer_lanes, refill_lanes, chunk, stack_depth, branching)
    _check(lib().rsi_build(_ptr(V), V.shape[0], _ptr(T), T.shape[0], ctypes.byref(o), _stream(stream),
                           ctypes.byref(h)))
    return h


def rsi_rebuild(h, V, T, stream=None):
    V = _dev_f32(V, "V")
    T = _dev_i32(T, "T")
    _check(lib().rsi_rebuild(h, _ptr(V), V.shape[0], _ptr(T), _stream(stream)))


def rsi_refit(h, V, stream=None):
    V = _dev_f32(V, "V")
    _check(lib().rsi_refit(h, _ptr(V), V.shape[0], _stream(stream)))


def rsi_query(h, S, E, mode, out: rsi_outputs, stream=None):
    S = _dev_f32(S, "S")
    E = _dev_f32(E, "E")
    if S.shape != E.shape:
        raise ValueError("S and E must have the same shape")
    _check(lib().rsi_query(h, _ptr(S), _ptr(E), S.shape[0], mode, ctypes.byref(out), _stream(stream)))


def rsi_query_noalloc(h, S, E, mode, out: rsi_outputs, stream=None):
    """rsi_query without any device allocation (boolean, first-hit and count
    modes); the library's scratch is a fixed array per GPU."""
    S = _dev_f32(S, "S")
    E = _dev_f32(E, "E")
    if S.shape != E.shape:
        raise ValueError("S and E must have the same shape")
    _check(lib().rsi_query_noalloc(h, _ptr(S), _ptr(E), S.shape[0], mode, ctypes.byref(out), _stream(stream)))


def rsi_first_hit_backward(h, V, S, E, tri, g_t=None, g_uv=None, g_point=None, dV=None, dS=None, dE=None,
                           stream=None):
    """dV is accumulated (pass zeros); dS / dE are written.  Returns (dV, dS, dE)."""
    V = _dev_f32(V, "V")
    S = _dev_f32(S, "S")
    E = _dev_f32(E, "E")
    n = S.shape[0]
    if tri.dtype != torch.int32 or not tri.is_contiguous() or tri.numel() != n:
        raise TypeError("tri must be a contiguous int32 [n] tensor")
    for name, g, c in (("g_t", g_t, 1), ("g_uv", g_uv, 2), ("g_point", g_point, 3)):
        if g is not None and (g.dtype != torch.float32 or not g.is_contiguous() or g.numel() != c * n):
            raise TypeError(f"{name} must be a contiguous float32 tensor with {c} values per segment")
    if dV is None:
        dV = torch.zeros_like(V)
    if dS is None:
        dS = torch.empty_like(S)
    if dE is None:
        dE = torch.empty_like(E)
    _check(lib().rsi_first_hit_backward(h, _ptr(V), V.shape[0], _ptr(S), _ptr(E), n, _ptr(tri), _ptr(g_t), _ptr(g_uv),
                                        _ptr(g_point), _ptr(dV), _ptr(dS), _ptr(dE), _stream(stream)))
    return dV, dS, dE


def rsi_segment_order(h, S, E, order, stream=None):
    _check(lib().rsi_segment_order(h, _ptr(S), _ptr(E), S.shape[0], _ptr(order), _stream(stream)))


def rsi_gather_segments(h, S, E, order, S_out, E_out, stream=None):
    _check(lib().rsi_gather_segments(h, _ptr(S), _ptr(E), _ptr(order), S.shape[0], _ptr(S_out), _ptr(E_out),
                                     _stream(stream)))


def rsi_compact(h, n_r, ids, hit=None, tri=None, t=None, point=None, S=None, E=None, dist=None, tri_out=None,
                point_out=None, stream=None):
    n = ctypes.c_int64()
    _check(lib().rsi_compact(h, _ptr(hit), _ptr(tri), _ptr(t), _ptr(point), _ptr(S), _ptr(E), n_r, _ptr(ids),
                             _ptr(dist), _ptr(tri_out), _ptr(point_out), ctypes.byref(n), _stream(stream)))
    return n.value


def rsi_inside(h, P, inside, count=None, E=None, stream=None):
    _check(lib().rsi_inside(h, _ptr(P), P.shape[0], _ptr(inside), _ptr(count), _ptr(E), _stream(stream)))


def rsi_spill_info(h):
    a, b = ctypes.c_int64(), ctypes.c_int64()
    _check(lib().rsi_spill_info(h, ctypes.byref(a), ctypes.byref(b)))
    return a.value, b.value


def rsi_spill_read(h, seg, offset, count, ids, ts, stream=None):
    _check(lib().rsi_spill_read(h, _ptr(seg), _ptr(offset), _ptr(count), _ptr(ids), _ptr(ts),
                                _stream(stream)))


def rsi_query_stats(h, check=True):
    """Wait for the handle's last call and return its device-side state as a
    dict (rsi_stats); with check=True a failing status raises RsiError."""
    st = rsi_stats()
    status = lib().rsi_query_stats(h, ctypes.byref(st))
    if check:
        _check(status)
    d = {name: getattr(st, name) for name, _ in rsi_stats._fields_ if name != "reserved"}
    d["status"] = status
    return d


def read_spill(h, stream=None, device=None):
    """The overflow table and pool of the last all-hits query as tensors,
    void entries (walks handed to the deep pass) dropped."""
    nseg, ntot = rsi_spill_info(h)
    dev = device or torch.device("cuda", torch.cuda.current_device())
    sp = {"seg": torch.empty(nseg, dtype=torch.int32, device=dev),
          "offset": torch.empty(nseg, dtype=torch.int64, device=dev),
          "count": torch.empty(nseg, dtype=torch.int32, device=dev),
          "ids": torch.empty(ntot, dtype=torch.int32, device=dev),
          "ts": torch.empty(ntot, dtype=torch.float32, device=dev)}
    if nseg:
        rsi_spill_read(h, sp["seg"], sp["offset"], sp["count"], sp["ids"], sp["ts"], stream)
        keep = sp["count"] >= 0
        for k in ("seg", "offset", "count"):
            sp[k] = sp[k][keep]
    return sp


def rsi_set_counting(h, enable: bool):
    _check(lib().rsi_set_counting(h, 1 if enable else 0))


def rsi_get_counters(h):
    c = rsi_counters()
    _check(lib().rsi_get_counters(h, ctypes.byref(c)))
    return {name: getattr(c, name) for name, _ in rsi_counters._fields_}


def rsi_get_tree_info(h):
    t = rsi_tree_info()
    _check(lib().rsi_get_tree_info(h, ctypes.byref(t)))
    return {"n_t": t.n_t, "n_nodes": t.n_nodes, "height": t.height, "leaf_size": t.leaf_size,
            "entry": t.entry, "n_meshes": t.n_meshes}


def rsi_get_mesh_info(h, mesh):
    off, n, ht = ctypes.c_int64(), ctypes.c_int64(), ctypes.c_int32()
    _check(lib().rsi_get_mesh_info(h, mesh, ctypes.byref(off), ctypes.byref(n), ctypes.byref(ht)))
    return {"tri_offset": off.value, "n_t": n.value, "height": ht.value}


def rsi_export_tree(h):
    import numpy as np
    info = rsi_get_tree_info(h)
    n = info["n_nodes"]
    boxes = np.zeros((max(n, 1), 12), np.float32)
    refs = np.zeros((max(n, 1), 2), np.int32)
    order = np.zeros(max(info["n_t"], 1), np.int32)
    keys = np.zeros(max(info["n_t"], 1), np.uint64)
    P = ctypes.c_void_p
    _check(lib().rsi_export_tree(h, boxes.ctypes.data_as(P), refs.ctypes.data_as(P),
                                 order.ctypes.data_as(P), keys.ctypes.data_as(P)))
    return {"boxes": boxes[:n], "refs": refs[:n], "order": order[:info["n_t"]], "keys": keys[:info["n_t"]],
            **info}


OPT_FIELDS = ("leaf_size", "block_size", "defer_lanes", "refill_lanes", "chunk", "stack_depth", "branching")


def make_opts(d=None):
    d = d or {}
    return rsi_opts(*[int(d.get(k, 0)) for k in OPT_FIELDS])


def rsi_set_opts(h, **opts):
    o = make_opts(opts)
    _check(lib().rsi_set_opts(h, ctypes.byref(o)))


def rsi_get_opts(h):
    o = rsi_opts()
    _check(lib().rsi_get_opts(h, ctypes.byref(o)))
    return {k: getattr(o, k) for k in OPT_FIELDS}


def rsi_tune(h, job, candidates, reps=5, stream=None):
    """Time each candidate (list of option dicts) on `job`, apply the fastest.
    Returns (best index, list of median milliseconds)."""
    cand = (rsi_opts * len(candidates))(*[make_opts(c) for c in candidates])
    ms = (ctypes.c_float * len(candidates))()
    best = ctypes.c_int32()
    _check(lib().rsi_tune(h, ctypes.byref(job), ctypes.cast(cand, ctypes.c_void_p), len(candidates), reps,
                          ctypes.cast(ms, ctypes.c_void_p), ctypes.byref(best), _stream(stream)))
    return best.value, list(ms)


def rsi_destroy(h):
    if h:
        lib().rsi_destroy(h)


# ---------------------------------------------------------------- helpers --

def parse_mode(mode) -> int:
    if isinstance(mode, int):
        return mode
    m = 0
    for part in str(mode).replace("+", "|").split("|"):
        m |= MODE_NAMES[part.strip()]
    return m


class Mesh:
    """A BVH over a triangle mesh on the current HIP device."""

    def __init__(self, V, T, leaf_size=0, block_size=0, stream=None, defer_lanes=0, refill_lanes=0,
                 chunk=0, stack_depth=0, branching=0, check=True):
        self.handle = None
        self.V = V
        self.T = T
        self.n_t = T.shape[0]
        self.n_v = V.shape[0]
        self.handle = rsi_build(V, T, leaf_size, block_size, stream, defer_lanes, refill_lanes, chunk,
                                stack_depth, branching)
        if check:
            # the build is asynchronous: wait once here so that bad triangle
            # indices raise at construction
            try:
                rsi_query_stats(self.handle)
            except RsiError:
                self.close()
                raise

    def _check_v(self, V):
        if V.shape[0] != self.n_v:
            raise ValueError(f"V has {V.shape[0]} vertices; the mesh was built with {self.n_v}")

    def rebuild(self, V, T, stream=None):
        if T.shape[0] != self.n_t:
            raise ValueError(f"T has {T.shape[0]} triangles; the mesh was built with {self.n_t}")
        rsi_rebuild(self.handle, V, T, stream)
        self.n_v = V.shape[0]

    def refit(self, V, stream=None):
        self._check_v(V)
        rsi_refit(self.handle, V, stream)

    def stats(self, check=True):
        """Wait for the last call and return its device-side state (rsi_stats)."""
        return rsi_query_stats(self.handle, check)

    def alloc_outputs(self, n_r, mode, capacity=4, device=None):
        mode = parse_mode(mode)
        dev = device or torch.device("cuda", torch.cuda.current_device())
        out = {}
        if mode & RSI_BOOL:
            out["hit"] = torch.empty(n_r, dtype=torch.uint8, device=dev)
        if mode & RSI_FIRST_HIT:
            out["tri"] = torch.empty(n_r, dtype=torch.int32, device=dev)
            out["t"] = torch.empty(n_r, dtype=torch.float32, device=dev)
            out["uv"] = torch.empty(n_r, 2, dtype=torch.float32, device=dev)
            out["point"] = torch.empty(n_r, 3, dtype=torch.float32, device=dev)
        if mode & (RSI_ALL_HITS | RSI_COUNT):
            out["count"] = torch.empty(n_r, dtype=torch.int32, device=dev)
        if mode & RSI_ALL_HITS:
            out["ids"] = torch.empty(n_r, capacity, dtype=torch.int32, device=dev)
            out["ts"] = torch.empty(n_r, capacity, dtype=torch.float32, device=dev)
        return out

    @staticmethod
    def outputs_struct(out, capacity=4):
        sp_ids, sp_ts = out.get("spill_ids"), out.get("spill_ts")
        return rsi_outputs(_ptr(out.get("hit")), _ptr(out.get("tri")), _ptr(out.get("t")),
                           _ptr(out.get("uv")), _ptr(out.get("point")), _ptr(out.get("count")),
                           _ptr(out.get("ids")), _ptr(out.get("ts")), capacity, 0, _ptr(out.get("spill_off")),
                           _ptr(sp_ids), _ptr(sp_ts), 0 if sp_ids is None else sp_ids.numel())

    def query_into(self, S, E, mode, out, capacity=4, stream=None):
        rsi_query(self.handle, S, E, parse_mode(mode), self.outputs_struct(out, capacity), stream)
        return out

    def query_noalloc_into(self, S, E, mode, out, stream=None):
        """rsi_query_noalloc into caller-allocated outputs (see alloc_outputs)."""
        rsi_query_noalloc(self.handle, S, E, parse_mode(mode), self.outputs_struct(out), stream)
        return out

    def query(self, S, E, mode="bool", capacity=4, stream=None):
        """Allocate outputs and query.  With all hits, wait for the query:
        if the library's spill pool was too small (RSI_E_OVERFLOW), query
        again (the pool has grown to fit), then read the overflowed
        segments' full lists into out["spill"]."""
        mode = parse_mode(mode)
        out = self.alloc_outputs(S.shape[0], mode, capacity, S.device)
        self.query_into(S, E, mode, out, capacity, stream)
        if mode & RSI_ALL_HITS:
            st = rsi_query_stats(self.handle, check=False)
            if st["status"] == RSI_E_OVERFLOW:
                self.query_into(S, E, mode, out, capacity, stream)
                st = rsi_query_stats(self.handle, check=False)
            _check(st["status"])
            if st["overflow_segments"]:
                out["spill"] = read_spill(self.handle, stream, S.device)
        return out

    def barycentric(self, S, E, stream=None):
        """The paper's `barycentric` output (Section 2.4): intersecting rays,
        distances, intersecting triangles, intersecting points, for the
        segments that cross the mesh (first hit of each)."""
        r = self.query(S, E, "first", stream=stream)
        n = S.shape[0]
        dev = S.device
        ids = torch.empty(n, dtype=torch.int32, device=dev)
        dist = torch.empty(n, dtype=torch.float32, device=dev)
        tri = torch.empty(n, dtype=torch.int32, device=dev)
        pts = torch.empty(n, 3, dtype=torch.float32, device=dev)
        k = rsi_compact(self.handle, n, ids, tri=r["tri"], t=r["t"], point=r["point"], S=S, E=E, dist=dist,
                        tri_out=tri, point_out=pts, stream=stream)
        return {"intersecting_rays": ids[:k], "distances": dist[:k], "intersecting_triangles": tri[:k],
                "intersecting_points": pts[:k]}

    def segment_order(self, S, E, stream=None):
        """Morton order of the segments (octant of the direction, then the
        midpoint's 30-bit code) and the segments gathered into it."""
        S, E = _dev_f32(S, "S"), _dev_f32(E, "E")
        order = torch.empty(S.shape[0], dtype=torch.int32, device=S.device)
        rsi_segment_order(self.handle, S, E, order, stream)
        So, Eo = torch.empty_like(S), torch.empty_like(E)
        rsi_gather_segments(self.handle, S, E, order, So, Eo, stream)
        return order, So, Eo

    def crossing_ids(self, hit, stream=None):
        """Ids of the segments whose boolean output is set, in order."""
        ids = torch.empty(hit.shape[0], dtype=torch.int32, device=hit.device)
        k = rsi_compact(self.handle, hit.shape[0], ids, hit=hit, stream=stream)
        return ids[:k]

    def inside(self, P, stream=None):
        """Odd-parity inside test of points P [n, 3]: returns inside (uint8),
        the crossing counts and the far segment ends used."""
        P = _dev_f32(P, "P")
        n = P.shape[0]
        out = {"inside": torch.empty(n, dtype=torch.uint8, device=P.device),
               "count": torch.empty(n, dtype=torch.int32, device=P.device),
               "E": torch.empty(n, 3, dtype=torch.float32, device=P.device)}
        rsi_inside(self.handle, P, out["inside"], out["count"], out["E"], stream)
        return out

    def first_hit_backward(self, V, S, E, tri, g_t=None, g_uv=None, g_point=None, stream=None):
        self._check_v(V)
        return rsi_first_hit_backward(self.handle, V, S, E, tri, g_t, g_uv, g_point, stream=stream)

    def set_counting(self, enable=True):
        rsi_set_counting(self.handle, enable)

    def set_opts(self, **opts):
        rsi_set_opts(self.handle, **opts)

    def opts(self):
        return rsi_get_opts(self.handle)

    def tune(self, S, E, mode, candidates, capacity=4, reps=5, stream=None):
        """Autotune on a real query of (S, E); the fastest candidate stays applied."""
        mode = parse_mode(mode)
        out = self.alloc_outputs(S.shape[0], mode, capacity, S.device)
        o = self.outputs_struct(out, capacity)
        job = rsi_tune_job(_ptr(self.V), self.V.shape[0], _ptr(self.T), _ptr(_dev_f32(S, "S")),
                           _ptr(_dev_f32(E, "E")), S.shape[0], ctypes.cast(ctypes.pointer(o), ctypes.c_void_p),
                           None, None, None, None, mode, 0)
        return rsi_tune(self.handle, job, candidates, reps, stream)

    def counters(self):
        return rsi_get_counters(self.handle)

    def tree(self):
        return rsi_export_tree(self.handle)

    def tree_info(self):
        return rsi_get_tree_info(self.handle)

    def close(self):
        if self.handle:
            rsi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def _ptr_array(tensors):
    arr = (ctypes.c_void_p * len(tensors))(*[t.data_ptr() if t is not None and t.numel() else 0
                                             for t in tensors])
    return arr


class Batch:
    """Many meshes in one handle: one build launch per stage for all of them,
    one persistent query launch over every (mesh, segment) item, and an
    optional HIP graph of rebuild + query replayed with one launch."""

    def __init__(self, meshes, leaf_size=0, block_size=0, stream=None, defer_lanes=0, refill_lanes=0, chunk=0,
                 stack_depth=0, branching=0, check=True):
        self.handle = None
        self.meshes = [(_dev_f32(V, "V"), _dev_i32(T, "T")) for V, T in meshes]
        M = len(self.meshes)
        self._V = _ptr_array([V for V, _ in self.meshes])
        self._T = _ptr_array([T for _, T in self.meshes])
        self._nv = (ctypes.c_int64 * M)(*[V.shape[0] for V, _ in self.meshes])
        self._nt = (ctypes.c_int64 * M)(*[T.shape[0] for _, T in self.meshes])
        o = rsi_opts(leaf_size, block_size, defer_lanes, refill_lanes, chunk, stack_depth, branching)
        h = ctypes.c_void_p()
        _check(lib().rsi_batch_create(M, ctypes.cast(self._V, ctypes.c_void_p), ctypes.cast(self._nv, ctypes.c_void_p),
                                      ctypes.cast(self._T, ctypes.c_void_p), ctypes.cast(self._nt, ctypes.c_void_p),
                                      ctypes.byref(o), _stream(stream), ctypes.byref(h)))
        self.handle = h
        self._keep = None
        self._graph_keep = None
        if check:
            # the build is asynchronous: wait once so bad indices raise here
            try:
                rsi_query_stats(self.handle)
            except RsiError:
                self.close()
                raise

    @property
    def n_meshes(self):
        return len(self.meshes)

    def rebuild(self, stream=None):
        _check(lib().rsi_batch_rebuild(self.handle, _stream(stream)))

    def alloc_outputs(self, segments, mode, capacity=4):
        mode = parse_mode(mode)
        outs = []
        for S, _ in segments:
            n = S.shape[0]
            d = {}
            if mode & RSI_ALL_HITS:
                d["count"] = torch.empty(n, dtype=torch.int32, device=S.device)
                d["ids"] = torch.empty(n, capacity, dtype=torch.int32, device=S.device)
                d["ts"] = torch.empty(n, capacity, dtype=torch.float32, device=S.device)
            if mode & RSI_BOOL:
                d["hit"] = torch.empty(n, dtype=torch.uint8, device=S.device)
            if mode & RSI_FIRST_HIT:
                d["tri"] = torch.empty(n, dtype=torch.int32, device=S.device)
                d["t"] = torch.empty(n, dtype=torch.float32, device=S.device)
                d["uv"] = torch.empty(n, 2, dtype=torch.float32, device=S.device)
                d["point"] = torch.empty(n, 3, dtype=torch.float32, device=S.device)
            outs.append(d)
        return outs

    def _tables(self, segments, mode, outs, keep="_keep"):
        if len(segments) != self.n_meshes or len(outs) != self.n_meshes:
            raise ValueError("one (S, E) pair and one output dict per mesh")
        segs = [(_dev_f32(S, "S"), _dev_f32(E, "E")) for S, E in segments]
        S = _ptr_array([s for s, _ in segs])
        E = _ptr_array([e for _, e in segs])
        n = (ctypes.c_int64 * self.n_meshes)(*[s.shape[0] for s, _ in segs])
        cap = lambda d: d["ids"].shape[1] if "ids" in d else 1
        o = (rsi_outputs * self.n_meshes)(*[Mesh.outputs_struct(d, cap(d)) for d in outs])
        setattr(self, keep, (segs, outs, S, E, n, o))  # buffers the launch (or graph) refers to
        c = lambda x: ctypes.cast(x, ctypes.c_void_p)
        return c(S), c(E), c(n), parse_mode(mode), c(o)

    def query_into(self, segments, mode, outs, stream=None):
        S, E, n, m, o = self._tables(segments, mode, outs)
        _check(lib().rsi_batch_query(self.handle, S, E, n, m, o, _stream(stream)))
        return outs

    def query(self, segments, mode="bool", capacity=4, stream=None):
        """Allocate outputs and run one batched query.  With all hits, wait
        for it, query again if the spill pool was too small, and return the
        overflowed work items' full lists as outs[0]["spill"] (its `seg` is
        the work item: the offset of the mesh's segments plus the index)."""
        m = parse_mode(mode)
        outs = self.alloc_outputs(segments, m, capacity)
        self.query_into(segments, m, outs, stream)
        if m & RSI_ALL_HITS:
            st = rsi_query_stats(self.handle, check=False)
            if st["status"] == RSI_E_OVERFLOW:
                self.query_into(segments, m, outs, stream)
                st = rsi_query_stats(self.handle, check=False)
            _check(st["status"])
            if st["overflow_segments"]:
                outs[0]["spill"] = read_spill(self.handle, stream, segments[0][0].device)
        return outs

    def stats(self, check=True):
        return rsi_query_stats(self.handle, check)

    def capture(self, segments, mode, outs, rebuild=True, stream=None):
        # the graph keeps its own tables on the device; keep its buffers alive here
        S, E, n, m, o = self._tables(segments, mode, outs, keep="_graph_keep")
        _check(lib().rsi_batch_capture(self.handle, S, E, n, m, o, 1 if rebuild else 0, _stream(stream)))

    def replay(self, stream=None):
        _check(lib().rsi_batch_replay(self.handle, _stream(stream)))

    def mesh_info(self, m):
        return rsi_get_mesh_info(self.handle, m)

    def set_opts(self, **opts):
        rsi_set_opts(self.handle, **opts)

    def opts(self):
        return rsi_get_opts(self.handle)

    def tune(self, segments, mode, candidates, reps=5, stream=None):
        """Autotune the batched query of `segments`; the fastest candidate stays applied."""
        outs = self.alloc_outputs(segments, mode)
        S, E, n, m, o = self._tables(segments, mode, outs)
        job = rsi_tune_job(None, 0, None, None, None, 0, None, S, E, n, o, m, 0)
        return rsi_tune(self.handle, job, candidates, reps, stream)

    def tree(self):
        return rsi_export_tree(self.handle)

    def close(self):
        if self.handle:
            rsi_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class FirstHit(torch.autograd.Function):
    """Differentiable first hit of segments (S, E) against a mesh with
    learnable vertices V (the topology T is fixed by `mesh`).

    forward(V, S, E, mesh) -> (t [n], uv [n, 2], point [n, 3], tri [n])
    The forward refits `mesh` to V (bounds only, same tree topology) and runs
    the first-hit query; the backward runs the library's adjoint kernel and
    returns dL/dV, dL/dS, dL/dE (tri is not differentiable).
    """

    @staticmethod
    def forward(ctx, V, S, E, mesh):
        mesh._check_v(V)
        V = V.detach().contiguous()
        S = S.detach().contiguous()
        E = E.detach().contiguous()
        mesh.refit(V)
        out = mesh.query(S, E, "first")
        ctx.mesh = mesh
        ctx.save_for_backward(V, S, E, out["tri"])
        ctx.mark_non_differentiable(out["tri"])
        return out["t"], out["uv"], out["point"], out["tri"]

    @staticmethod
    def backward(ctx, g_t, g_uv, g_point, g_tri):
        V, S, E, tri = ctx.saved_tensors
        f = lambda g: None if g is None else g.contiguous().to(torch.float32)
        dV, dS, dE = rsi_first_hit_backward(ctx.mesh.handle, V, S, E, tri, f(g_t), f(g_uv), f(g_point))
        return dV, dS, dE, None


def first_hit(V, S, E, mesh):
    """Convenience wrapper of FirstHit.apply."""
    return FirstHit.apply(V, S, E, mesh)
