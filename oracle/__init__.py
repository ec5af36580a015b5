"""FP64 brute-force oracle for segment / triangle-mesh crossing queries.

TEST INFRASTRUCTURE ONLY: imported by the tests, the smoke check and the
benchmark's CPU-baseline leg, never by the library.  The arithmetic lives in
`rsi_oracle.c` (plain C, OpenMP over segments); this module only compiles it
with gcc and marshals numpy arrays.  It shares no code with the GPU path.

Functions
  query(V, T, S, E, cap=0, threads=0) -> dict of numpy arrays
      count, first_tri, first_tuv (t, u, v), first_p, list_tri, list_t
  degenerate(V, T, S, E, delta, threads=0) -> uint8 flags per segment
      bit 1 edge within delta, bit 2 endpoint within delta of a triangle,
      bit 4 two crossings within delta of each other along the segment
  first_hit_grad(V, T, S, E, tri, tuv, g_t, g_uv, g_p, with_abs) -> dV, dS, dE
      (FP64; with_abs also returns the per-element sum of |contributions|)
  seg_seg_dist, pt_tri_dist: the distance routines the classifier uses
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "rsi_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = False) -> str:
    """Compile rsi_oracle.c into liboracle.so with gcc -O2 -fopenmp."""
    if force or not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        tmp = _LIB_PATH + ".tmp%d" % os.getpid()
        cmd = ["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c11",
               "-Wall", "-Wno-unknown-pragmas", "-o", tmp, _SRC, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    build()
    lib = ctypes.CDLL(_LIB_PATH)
    P = ctypes.c_void_p
    i64 = ctypes.c_int64
    i32 = ctypes.c_int32
    lib.rsi_oracle_query.argtypes = [P, i64, P, i64, P, P, i64, i32, P, P, P, P, P, P, i32]
    lib.rsi_oracle_query.restype = ctypes.c_int
    lib.rsi_oracle_degenerate.argtypes = [P, i64, P, i64, P, P, i64, ctypes.c_double, P, i32]
    lib.rsi_oracle_degenerate.restype = ctypes.c_int
    lib.rsi_oracle_first_hit_grad.argtypes = [P, i64, P, i64, P, P, i64, P, P, P, P, P, P, P, P, P]
    lib.rsi_oracle_first_hit_grad.restype = ctypes.c_int
    lib.rsi_oracle_seg_seg_dist.argtypes = [P, P, P, P]
    lib.rsi_oracle_seg_seg_dist.restype = ctypes.c_double
    lib.rsi_oracle_pt_tri_dist.argtypes = [P, P, P, P]
    lib.rsi_oracle_pt_tri_dist.restype = ctypes.c_double
    lib.rsi_oracle_max_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _c(a, dtype):
    return np.ascontiguousarray(a, dtype=dtype)


def _mesh_args(V, T, S, E):
    # FP32 inputs promote exactly to FP64; FP64 inputs pass through unchanged
    return (_c(V, np.float64).reshape(-1, 3), _c(T, np.int32).reshape(-1, 3),
            _c(S, np.float64).reshape(-1, 3), _c(E, np.float64).reshape(-1, 3))


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def max_threads() -> int:
    return int(_load().rsi_oracle_max_threads())


def query(V, T, S, E, cap: int = 0, threads: int = 0) -> dict:
    lib = _load()
    V, T, S, E = _mesh_args(V, T, S, E)
    nr = S.shape[0]
    out = {
        "count": np.zeros(nr, np.int32),
        "first_tri": np.zeros(nr, np.int32),
        "first_tuv": np.zeros((nr, 3), np.float64),
        "first_p": np.zeros((nr, 3), np.float64),
    }
    if cap > 0:
        out["list_tri"] = np.zeros((nr, cap), np.int32)
        out["list_t"] = np.zeros((nr, cap), np.float64)
    rc = lib.rsi_oracle_query(_p(V), V.shape[0], _p(T), T.shape[0], _p(S), _p(E), nr, int(cap),
                              _p(out["count"]), _p(out["first_tri"]), _p(out["first_tuv"]),
                              _p(out["first_p"]), _p(out.get("list_tri")), _p(out.get("list_t")),
                              int(threads))
    if rc != 0:
        raise ValueError("triangle index out of range")
    out["hit"] = (out["count"] > 0).astype(np.uint8)
    return out


def degenerate(V, T, S, E, delta: float, threads: int = 0) -> np.ndarray:
    lib = _load()
    V, T, S, E = _mesh_args(V, T, S, E)
    flags = np.zeros(S.shape[0], np.uint8)
    rc = lib.rsi_oracle_degenerate(_p(V), V.shape[0], _p(T), T.shape[0], _p(S), _p(E),
                                   S.shape[0], float(delta), _p(flags), int(threads))
    if rc != 0:
        raise ValueError("triangle index out of range")
    return flags


def first_hit_grad(V, T, S, E, tri, tuv, g_t=None, g_uv=None, g_p=None, with_abs=False):
    lib = _load()
    V, T, S, E = _mesh_args(V, T, S, E)
    nr = S.shape[0]
    tri = _c(tri, np.int32)
    tuv = _c(tuv, np.float64).reshape(-1, 3)
    g_t = None if g_t is None else _c(g_t, np.float64).reshape(nr)
    g_uv = None if g_uv is None else _c(g_uv, np.float64).reshape(nr, 2)
    g_p = None if g_p is None else _c(g_p, np.float64).reshape(nr, 3)
    dV = np.zeros((V.shape[0], 3), np.float64)
    dS = np.zeros((nr, 3), np.float64)
    dE = np.zeros((nr, 3), np.float64)
    dV_abs = np.zeros((V.shape[0], 3), np.float64) if with_abs else None
    rc = lib.rsi_oracle_first_hit_grad(_p(V), V.shape[0], _p(T), T.shape[0], _p(S), _p(E), nr,
                                       _p(tri), _p(tuv), _p(g_t), _p(g_uv), _p(g_p),
                                       _p(dV), _p(dS), _p(dE), _p(dV_abs))
    if rc != 0:
        raise ValueError("triangle index out of range")
    if with_abs:
        return dV, dS, dE, dV_abs
    return dV, dS, dE


def seg_seg_dist(p1, q1, p2, q2) -> float:
    a = [_c(x, np.float64) for x in (p1, q1, p2, q2)]
    return float(_load().rsi_oracle_seg_seg_dist(*[_p(x) for x in a]))


def pt_tri_dist(p, a, b, c) -> float:
    v = [_c(x, np.float64) for x in (p, a, b, c)]
    return float(_load().rsi_oracle_pt_tri_dist(*[_p(x) for x in v]))
