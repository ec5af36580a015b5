"""Benchmark: segments/s against a ~30k-triangle mesh on one MI355X.

Workload: the 123 x 123 value-noise heightfield (29,768 triangles, 1e-3 xy
jitter) and 10M segments (start uniform in the mesh box, direction uniform on
the sphere, length log-uniform in [0.01, 1]), all synthetic and seeded.  This
stands in for the paper's unpublished 29,284-triangle surface with 10M random
rays (Section 2, Table 1; Section 4.1, Table 3).

One step = one pass of the whole path on that batch: rebuild the BVH from the
mesh (centroids, Morton codes, radix sort, hierarchy with bottom-up bounds)
and answer the boolean query for all 10M segments.  Inputs are resident in
HBM before timing starts.  `value` = segments per second of that step.

Also reported: the query alone in boolean and all-hits (capacity 4) modes,
the build alone, the dominant kernel's average duration (HIP events on the
launch stream) with its ALU roofline, and the FP64 oracle timed on the host's
cores on a bounded sample (a baseline, not the target).
"""
from __future__ import annotations

import argparse
import json
import os
import platform
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# VALU lane-operations per unit of work, counted from the kernel source
# (rsi_device.h): one segment / box slab test and one Moller-Trumbore test.
OPS_PER_BOX_TEST = 26
OPS_PER_TRI_TEST = 45
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one VALU lane-op per lane per clock;
# packed FP32 is not used)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-r", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the segment queries of this library run on a single "
              "device (multi-GPU sharding is a design note, not built); use --gpus 1", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2209_02878_amd import rsi
    from paper_2209_02878_amd import workloads as wl

    assert torch.cuda.is_available(), "bench.py needs a GPU"
    dev = torch.device("cuda", 0)
    torch.cuda.set_device(dev)
    t0 = time.time()
    w = wl.config2(n_r=args.n_r)
    log(f"workload {w.name}: n_t={w.n_t} n_v={w.n_v} n_r={w.n_r} generated in {time.time() - t0:.1f}s")
    V = torch.from_numpy(w.V).to(dev)
    T = torch.from_numpy(w.T).to(dev)
    S = torch.from_numpy(w.S).to(dev)
    E = torch.from_numpy(w.E).to(dev)
    stream = torch.cuda.current_stream()

    mesh = rsi.Mesh(V, T)
    info = mesh.tree_info()
    out_b = mesh.alloc_outputs(w.n_r, "bool")
    out_a = mesh.alloc_outputs(w.n_r, "all", capacity=4)
    torch.cuda.synchronize()

    def step():
        mesh.rebuild(V, T)
        mesh.query_into(S, E, "bool", out_b)

    for _ in range(args.warmup):
        step()
    torch.cuda.synchronize()
    t_start = time.perf_counter()
    for _ in range(args.steps):
        step()
    torch.cuda.synchronize()
    elapsed = time.perf_counter() - t_start
    ms_per_step = 1e3 * elapsed / args.steps
    value = w.n_r / (ms_per_step / 1e3) / 1e6
    log(f"step (rebuild + bool query): {ms_per_step:.3f} ms -> {value:.1f} Msegments/s")

    # ---- dominant kernel: the boolean query launch, timed with HIP events
    def time_events(fn, reps):
        evs = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)) for _ in range(reps)]
        for a, b in evs:
            a.record(stream)
            fn()
            b.record(stream)
        torch.cuda.synchronize()
        return [a.elapsed_time(b) for a, b in evs]

    reps = max(args.steps, 10)
    q_bool = time_events(lambda: mesh.query_into(S, E, "bool", out_b), reps)
    q_all = time_events(lambda: mesh.query_into(S, E, "all", out_a, capacity=4), max(5, reps // 2))
    b_only = time_events(lambda: mesh.rebuild(V, T), reps)
    kb = float(np.mean(q_bool))
    log(f"bool query kernel: mean {kb:.3f} ms, median {np.median(q_bool):.3f} ms; "
        f"all-hits query: median {np.median(q_all):.3f} ms; rebuild: median {np.median(b_only):.3f} ms")

    # ---- algorithmic work of that launch, from the counting variant (untimed)
    mesh.set_counting(True)
    mesh.query_into(S, E, "bool", out_b)
    torch.cuda.synchronize()
    cnt = mesh.counters()
    mesh.set_counting(False)
    ops = OPS_PER_BOX_TEST * cnt["box_tests"] + OPS_PER_TRI_TEST * cnt["tri_tests"]
    achieved_tops = ops / (kb / 1e3) / 1e12
    hits = int(out_b["hit"].sum().item())
    log(f"counters: {cnt}; hit fraction {hits / w.n_r:.4f}")

    rec = {
        "metric": "Msegments/s vs 30k-tri mesh (bool & all-hits); fwd+bwd vs fwd at 1e-5 rel err",
        "value": round(value, 3),
        "unit": "Msegments/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            "workload": "heightfield 123x123 (29,768 triangles, value noise, 1e-3 xy jitter), 10M segments "
                        "(start uniform in mesh box, direction uniform on sphere, length log-uniform [0.01,1]); "
                        "step = BVH rebuild + boolean query",
            "n_t": w.n_t, "n_r": w.n_r, "leaf_size": info["leaf_size"], "tree_height": info["height"],
        },
        "query_bool_ms": round(float(np.median(q_bool)), 4),
        "query_bool_msegments_per_s": round(w.n_r / np.median(q_bool) / 1e3, 2),
        "query_all_hits_k4_ms": round(float(np.median(q_all)), 4),
        "query_all_hits_k4_msegments_per_s": round(w.n_r / np.median(q_all) / 1e3, 2),
        "rebuild_ms": round(float(np.median(b_only)), 4),
        "hit_fraction": round(hits / w.n_r, 5),
        "work_per_segment": {"node_visits": cnt["node_visits"] / w.n_r, "box_tests": cnt["box_tests"] / w.n_r,
                             "tri_tests": cnt["tri_tests"] / w.n_r},
        "roofline": {
            "bound": "alu",
            "kernel": "k_query<bool>",
            "achieved": round(achieved_tops, 4),
            "peak": round(PEAK_VALU_TOPS, 3),
            "unit": "Tops/s",
            "frac": round(achieved_tops / PEAK_VALU_TOPS, 5),
            "traffic": None,
            "ops_per_launch": int(ops),
            "kernel_ms": round(kb, 4),
            "hbm_gbs_algorithmic": round(25.0 * w.n_r / (kb / 1e3) / 1e9, 2),
        },
    }

    # ---- CPU baseline: the FP64 oracle on a bounded sample, on the host cores
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        probe = 4000
        t1 = time.perf_counter()
        oracle.query(w.V, w.T, w.S[:probe], w.E[:probe])
        dt = time.perf_counter() - t1
        n_s = int(min(w.n_r, max(probe, probe * args.cpu_seconds / max(dt, 1e-6))))
        t1 = time.perf_counter()
        oracle.query(w.V, w.T, w.S[:n_s], w.E[:n_s])
        dt = time.perf_counter() - t1
        rec["cpu_baseline"] = {
            "value": round(n_s / dt / 1e6, 5),
            "unit": "Msegments/s",
            "cores": threads,
            "kind": "oracle",
            "sample": f"first {n_s} of the 10M segments against all 29,768 triangles, FP64 brute force "
                      f"over every pair, {dt:.1f} s",
            "cpu": platform.processor() or platform.machine(),
        }
        log(f"cpu baseline: {rec['cpu_baseline']}")
    mesh.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
