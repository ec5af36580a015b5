"""Command line and file I/O in the paper's formats (Section 2.3 to 2.5).

    python -m paper_2209_02878_amd.cli [vertices triangles rayFrom rayTo [silent|default] [barycentric|intercept_count]]

Inputs are the paper's four little-endian binary files: vertices (float32
x, y, z per vertex), triangles (int32 vertex indices, three per triangle),
rayFrom and rayTo (float32 segment starts and ends).  Without paths the
files `vertices_f32`, `triangles_i32`, `rayFrom_f32`, `rayTo_f32` under
`./input` are used.  The fifth argument `silent` suppresses the report (any
other value, e.g. `default`, keeps it); the sixth selects the output:

  (none)           crossing_detected_i32: int32 per segment, 1 if it crosses
  barycentric      intersecting_rays_i32, distances_f32,
                   intersecting_triangles_i32, intersecting_points_f32
                   (first hit of every crossing segment, in segment order;
                   distance = t |E - S|)
  intercept_count  num_intersections_i32: crossings per segment

The paper does not name its output files; these names and the output folder
(`--out`, default `./output`) are this library's.  Every step runs in the
HIP library; this module only reads and writes files.
"""
from __future__ import annotations

import argparse
import os
import sys
import time

import numpy as np

DEFAULT_NAMES = ("vertices_f32", "triangles_i32", "rayFrom_f32", "rayTo_f32")


def read_inputs(vertices: str, triangles: str, ray_from: str, ray_to: str):
    """Read the four binary input files; returns V, T, S, E (numpy)."""
    def load(path, dtype, what):
        a = np.fromfile(path, dtype=np.dtype(dtype).newbyteorder("<"))
        if a.size % 3:
            raise ValueError(f"{what} file {path}: {a.size} values is not a multiple of 3")
        return a.astype(dtype, copy=False).reshape(-1, 3)
    V = load(vertices, np.float32, "vertices")
    T = load(triangles, np.int32, "triangles")
    S = load(ray_from, np.float32, "rayFrom")
    E = load(ray_to, np.float32, "rayTo")
    if S.shape != E.shape:
        raise ValueError(f"rayFrom has {S.shape[0]} segments, rayTo {E.shape[0]}")
    return V, T, S, E


def write_inputs(folder: str, V, T, S, E) -> None:
    """Write arrays in the input format under the default names."""
    os.makedirs(folder, exist_ok=True)
    for name, a, dt in zip(DEFAULT_NAMES, (V, T, S, E), ("<f4", "<i4", "<f4", "<f4")):
        np.ascontiguousarray(a, dtype=dt).tofile(os.path.join(folder, name))


def run(V, T, S, E, mode: str = "default", device=None):
    """Run the query on the GPU; returns a dict of numpy arrays named as the
    output files (without the type suffix)."""
    import torch
    from . import rsi
    dev = device or torch.device("cuda", 0)
    t = lambda a, dt=torch.float32: torch.as_tensor(np.ascontiguousarray(a)).to(device=dev, dtype=dt)
    mesh = rsi.Mesh(t(V), t(T, torch.int32))
    Sd, Ed = t(S), t(E)
    try:
        if mode == "barycentric":
            r = mesh.barycentric(Sd, Ed)
            out = {"intersecting_rays": r["intersecting_rays"], "distances": r["distances"],
                   "intersecting_triangles": r["intersecting_triangles"],
                   "intersecting_points": r["intersecting_points"]}
        elif mode == "intercept_count":
            out = {"num_intersections": mesh.query(Sd, Ed, "count")["count"]}
        else:
            out = {"crossing_detected": mesh.query(Sd, Ed, "bool")["hit"].to(torch.int32)}
        torch.cuda.synchronize()
        return {k: v.cpu().numpy() for k, v in out.items()}
    finally:
        mesh.close()


SUFFIX = {"crossing_detected": "_i32", "num_intersections": "_i32", "intersecting_rays": "_i32",
          "distances": "_f32", "intersecting_triangles": "_i32", "intersecting_points": "_f32"}


def write_outputs(folder: str, results: dict) -> list:
    os.makedirs(folder, exist_ok=True)
    paths = []
    for k, a in results.items():
        p = os.path.join(folder, k + SUFFIX[k])
        dt = "<i4" if SUFFIX[k] == "_i32" else "<f4"
        np.ascontiguousarray(a, dtype=dt).tofile(p)
        paths.append(p)
    return paths


def parse_args(argv):
    ap = argparse.ArgumentParser(description=__doc__.split("\n")[0])
    ap.add_argument("files", nargs="*", help="vertices triangles rayFrom rayTo [silent|default] [mode]")
    ap.add_argument("--out", default="output")
    a = ap.parse_args(argv)
    files = list(a.files)
    if len(files) not in (0, 4, 5, 6):
        ap.error("expected 0 or 4 input files, then optionally silent|default and barycentric|intercept_count")
    paths = files[:4] if len(files) >= 4 else [os.path.join("input", n) for n in DEFAULT_NAMES]
    silent = len(files) >= 5 and files[4] == "silent"
    mode = files[5] if len(files) == 6 else "default"
    if mode not in ("default", "barycentric", "intercept_count"):
        ap.error(f"unknown output mode {mode!r}")
    return paths, silent, mode, a.out


def main(argv=None) -> int:
    paths, silent, mode, out = parse_args(sys.argv[1:] if argv is None else argv)
    t0 = time.perf_counter()
    V, T, S, E = read_inputs(*paths)
    t1 = time.perf_counter()
    res = run(V, T, S, E, mode)
    t2 = time.perf_counter()
    written = write_outputs(out, res)
    if not silent:
        print(f"{T.shape[0]} triangles, {S.shape[0]} segments; read {t1 - t0:.3f} s, "
              f"build + query {t2 - t1:.3f} s; wrote {', '.join(written)}")
    return 0


if __name__ == "__main__":
    sys.exit(main())
