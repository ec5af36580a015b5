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
# (rsi_device.h, query.hip): one slab test of an exact box (binary walk), one
# of a quantised box (four-way walk: each of the six planes is decoded with a
# byte conversion and an fma before the multiply) plus the per-node set-up
# of the four-way walk (exponent decode, corner offset, margin), and one
# Moller-Trumbore test.
OPS_PER_BOX_TEST = {2: 26, 4: 32}
OPS_PER_NODE = {2: 0, 4: 18}
OPS_PER_TRI_TEST = 45
# 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz (one VALU lane-op per lane per clock;
# packed FP32 is not used)
PEAK_VALU_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
PEAK_HBM_GBS = 8000.0


QUERY_SOURCES = ("paper_2209_02878_amd/csrc/query.hip", "paper_2209_02878_amd/csrc/rsi_device.h",
                 "paper_2209_02878_amd/csrc/rsi_host.h")
TRAFFIC_PROFILE = "profiles/hbm_traffic_k_query_heightfield29768_10Mseg.md"


def query_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in QUERY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per boolean-query launch from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by a copy of known size), or
    None when the kernel sources changed after those runs."""
    import re
    try:
        with open(os.path.join(ROOT, TRAFFIC_PROFILE)) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(r"^traffic-record: (.*)$", text, re.M)
    if not m:
        return None
    rec = dict(kv.split("=", 1) for kv in m.group(1).split())
    if rec.get("sources") != query_sources_hash():
        return None
    return (float(rec["fetch_kib"]) * float(rec["fetch_scale"]) +
            float(rec["write_kib"]) * float(rec["write_scale"])) * 1024.0


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def extra_workloads(torch, rsi, wl, dev, stream, time_events, log, w2, V2, T2, S2, E2):
    """The other configurations, reported beside the headline."""
    out = {}
    med = lambda xs: float(np.median(xs))

    # the headline mesh and segments: the binary walk, and Morton-ordered segments
    m = rsi.Mesh(V2, T2)
    ob = m.alloc_outputs(w2.n_r, "bool")
    oa = m.alloc_outputs(w2.n_r, "all", capacity=4)
    m.set_opts(branching=2)
    b2 = time_events(lambda: m.rebuild(V2, T2), 10)
    q2 = time_events(lambda: m.query_into(S2, E2, "bool", ob), 10)
    a2 = time_events(lambda: m.query_into(S2, E2, "all", oa, capacity=4), 5)
    out["heightfield_29768tri_10Mseg_binary_walk"] = {
        "rebuild_ms": round(med(b2), 4), "query_bool_ms": round(med(q2), 4),
        "query_all_hits_k4_ms": round(med(a2), 4)}
    log(f"binary walk: rebuild {med(b2):.3f} ms, bool {med(q2):.3f} ms, all-hits {med(a2):.3f} ms")
    m.set_opts(branching=4)
    order = torch.empty(w2.n_r, dtype=torch.int32, device=dev)
    So, Eo = torch.empty_like(S2), torch.empty_like(E2)
    oc = time_events(lambda: (rsi.rsi_segment_order(m.handle, S2, E2, order),
                              rsi.rsi_gather_segments(m.handle, S2, E2, order, So, Eo)), 5)
    qo = time_events(lambda: m.query_into(So, Eo, "bool", ob), 10)
    ao = time_events(lambda: m.query_into(So, Eo, "all", oa, capacity=4), 5)
    out["heightfield_29768tri_10Mseg_morton_ordered"] = {
        "order_and_gather_ms": round(med(oc), 4), "query_bool_ms": round(med(qo), 4),
        "query_all_hits_k4_ms": round(med(ao), 4)}
    log(f"ordered segments: order+gather {med(oc):.3f} ms, bool {med(qo):.3f} ms, all-hits {med(ao):.3f} ms")
    m.close()
    del ob, oa, order, So, Eo

    # closed 499,280-triangle sphere: all crossings (capacity 4) + first hit
    t0 = time.time()
    w = wl.config3()
    log(f"workload {w.name} generated in {time.time() - t0:.1f}s")
    V, T = torch.from_numpy(w.V).to(dev), torch.from_numpy(w.T).to(dev)
    S, E = torch.from_numpy(w.S).to(dev), torch.from_numpy(w.E).to(dev)
    m = rsi.Mesh(V, T)
    o = m.alloc_outputs(w.n_r, "all|first", capacity=4)
    b = time_events(lambda: m.rebuild(V, T), 5)
    q = time_events(lambda: m.query_into(S, E, "all|first", o, capacity=4), 5)
    nspill = rsi.rsi_spill_info(m.handle)[0]
    out["sphere_499280tri_10Mseg_all_first_k4"] = {
        "options": {k: m.opts()[k] for k in ("branching", "stack_depth")},
        "build_ms": round(med(b), 4), "query_ms": round(med(q), 4),
        "msegments_per_s": round(w.n_r / med(q) / 1e3, 2), "overflowed_segments": int(nspill)}
    log(f"sphere all|first: query {med(q):.3f} ms, build {med(b):.3f} ms, spill {nspill}")
    # odd-parity inside test of 10M points against the same closed surface
    P = torch.from_numpy(wl.inside_points(w.V, w.n_r, wl.seed_for(6, 1))).to(dev)
    ins = torch.empty(w.n_r, dtype=torch.uint8, device=dev)
    cnt = torch.empty(w.n_r, dtype=torch.int32, device=dev)
    ends = torch.empty(w.n_r, 3, dtype=torch.float32, device=dev)
    qi = time_events(lambda: rsi.rsi_inside(m.handle, P, ins, cnt, ends), 5)
    out["sphere_499280tri_10Mpoint_inside"] = {
        "ms": round(med(qi), 4), "mpoints_per_s": round(w.n_r / med(qi) / 1e3, 2),
        "inside_fraction": round(float(ins.float().mean().item()), 5)}
    log(f"inside test: {med(qi):.3f} ms for {w.n_r} points")
    m.close()
    del V, T, S, E, o, P, ins, cnt, ends

    # differentiable first hit: 199,712-triangle heightfield, 4M segments
    w = wl.config4()
    Vg, _ = wl.config4_target()
    V, T = torch.from_numpy(w.V).to(dev), torch.from_numpy(w.T).to(dev)
    S, E = torch.from_numpy(w.S).to(dev), torch.from_numpy(w.E).to(dev)
    n = 317
    gz = torch.from_numpy(Vg[:, 2].astype(np.float32)).to(dev)
    X = torch.clamp(S[:, 0] * (n - 1), 0, n - 1 - 1e-6)
    Y = torch.clamp(S[:, 1] * (n - 1), 0, n - 1 - 1e-6)
    i, j = X.long(), Y.long()
    a, c = X - i, Y - j
    k = j * n + i
    target = (gz[k] * (1 - a) * (1 - c) + gz[k + 1] * a * (1 - c) + gz[k + n] * (1 - a) * c
              + gz[k + n + 1] * a * c)
    m = rsi.Mesh(V, T)
    Vp = V.clone().requires_grad_(True)

    def fwd():
        with torch.no_grad():
            _, _, P, _ = rsi.FirstHit.apply(Vp, S, E, m)
            return ((P[:, 2] - target) ** 2).sum()

    def fwd_bwd():
        Vp.grad = None
        _, _, P, _ = rsi.FirstHit.apply(Vp, S, E, m)
        loss = ((P[:, 2] - target) ** 2).sum()
        loss.backward()

    f = time_events(fwd, 10)
    fb = time_events(fwd_bwd, 10)
    out["heightfield_199712tri_4Mseg_first_hit_grad"] = {
        "forward_ms": round(med(f), 4), "forward_backward_ms": round(med(fb), 4),
        "forward_msegments_per_s": round(w.n_r / med(f) / 1e3, 2),
        "forward_backward_msegments_per_s": round(w.n_r / med(fb) / 1e3, 2),
        "fwd_bwd_over_fwd_time": round(med(fb) / med(f), 3)}
    log(f"diff first hit: fwd {med(f):.3f} ms, fwd+bwd {med(fb):.3f} ms")
    m.close()
    del V, T, S, E, Vp

    # 64 meshes: one captured graph (rebuild all + one batched boolean query)
    # against 64 sequential plain calls (rebuild + query per mesh)
    t0 = time.time()
    ws = wl.config5()
    log(f"64-mesh batch generated in {time.time() - t0:.1f}s: {sum(x.n_t for x in ws)} triangles, "
        f"{sum(x.n_r for x in ws)} segments")
    meshes = [(torch.from_numpy(x.V).to(dev), torch.from_numpy(x.T).to(dev)) for x in ws]
    segs = [(torch.from_numpy(x.S).to(dev), torch.from_numpy(x.E).to(dev)) for x in ws]
    singles = [rsi.Mesh(Vm, Tm) for Vm, Tm in meshes]
    souts = [sm.alloc_outputs(Sm.shape[0], "bool") for sm, (Sm, _) in zip(singles, segs)]

    def sequential():
        for sm, (Vm, Tm), (Sm, Em), so in zip(singles, meshes, segs, souts):
            sm.rebuild(Vm, Tm)
            sm.query_into(Sm, Em, "bool", so)

    bt = rsi.Batch(meshes)
    bouts = bt.alloc_outputs(segs, "bool")
    bt.capture(segs, "bool", bouts, rebuild=True)
    seq = time_events(sequential, 3)
    rep = time_events(bt.replay, 10)
    torch.cuda.synchronize()
    same = all(torch.equal(bo["hit"], so["hit"]) for bo, so in zip(bouts, souts))
    ntot = sum(x.n_r for x in ws)
    out["batch_64_meshes_bool"] = {
        "n_t": int(sum(x.n_t for x in ws)), "n_r": int(ntot),
        "graph_replay_ms": round(med(rep), 4), "sequential_64_calls_ms": round(med(seq), 4),
        "graph_msegments_per_s": round(ntot / med(rep) / 1e3, 2),
        "speedup_vs_sequential": round(med(seq) / med(rep), 3), "identical_to_sequential": bool(same)}
    log(f"batch: graph {med(rep):.3f} ms vs sequential {med(seq):.3f} ms, identical={same}")
    bt.close()
    for sm in singles:
        sm.close()
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--n-r", type=int, default=10_000_000)
    ap.add_argument("--cpu-seconds", type=float, default=15.0, help="target length of the oracle baseline")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--headline-only", action="store_true",
                    help="only the 29,768-triangle step (for profiler runs)")
    ap.add_argument("--branching", type=int, default=0, choices=(0, 2, 4),
                    help="walk for the headline step: 4 = quantised four-way view (the default), 2 = binary tree")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="also run one 256 MiB device copy (known traffic for HBM counter scaling)")
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

    mesh = rsi.Mesh(V, T, branching=args.branching)
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
    br = mesh.opts()["branching"]
    ops = (OPS_PER_BOX_TEST[br] * cnt["box_tests"] + OPS_PER_NODE[br] * cnt["node_visits"] +
           OPS_PER_TRI_TEST * cnt["tri_tests"])
    achieved_tops = ops / (kb / 1e3) / 1e12
    hits = int(out_b["hit"].sum().item())
    log(f"counters: {cnt}; hit fraction {hits / w.n_r:.4f}")

    traffic = measured_traffic()
    traffic = None if traffic is None else round(traffic)
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
            "branching": mesh.opts()["branching"],
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
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "ops_per_launch": int(ops),
            "kernel_ms": round(kb, 4),
            "hbm_gbs_algorithmic": round(25.0 * w.n_r / (kb / 1e3) / 1e9, 2),
        },
    }

    if args.copy_calibration:
        x = torch.empty(64 * 1024 * 1024, dtype=torch.float32, device=dev)
        y = torch.empty_like(x)
        y.copy_(x)
        torch.cuda.synchronize()
        rec["copy_calibration_bytes"] = 2 * x.numel() * 4
        del x, y

    if not args.headline_only:
        mesh.close()
        rec["extra"] = extra_workloads(torch, rsi, wl, dev, stream, time_events, log, w, V, T, S, E)

    # ---- CPU baseline: the FP64 oracle on a bounded sample, on the host cores
    if not args.no_cpu_baseline:
        import oracle
        threads = oracle.max_threads()
        probe = 100_000
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
                      f"over every pair (box-overlap check, then the exact test), {dt:.1f} s",
            "cpu": platform.processor() or platform.machine(),
        }
        log(f"cpu baseline: {rec['cpu_baseline']}")
    if args.headline_only:
        mesh.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
