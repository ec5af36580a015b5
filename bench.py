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
launch stream) against the FP32 roofline (algorithmic FP32 operations of the
launch: 25 per child-box slab test and 50 per triangle test), its HBM traffic
and L2 hit rate from the committed counter profiles, the other workloads
(1,922-triangle heightfield, 499,280-triangle closed sphere with all hits,
differentiable first hit on 199,712 triangles, 64 meshes in one graph) and
the FP64 oracle timed on the host's cores (a baseline, not the target).
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# Algorithmic FP32 work per unit: a slab test of one child box (6 fma-class
# plane parameters counted as 2 ops each, 6 min/max, 4 reductions and
# clamps, 1 compare = 25) and a Moller-Trumbore triangle test (about 44 flops,
# 1 reciprocal, 6 compares = 50).  Counts of both come from the counting
# variant of the same launch.
OPS_PER_BOX_TEST = 25
OPS_PER_TRI_TEST = 50
# MI355X vector FP32: 157.3 TFLOP/s with packed (dual-issue) FP32, 78.6 without
PEAK_FP32_TFLOPS = 157.3
PEAK_FP32_TFLOPS_UNPACKED = 78.6
PEAK_HBM_GBS = 8000.0

# Paper figures quoted as context (Section 1; Tables 1 and 3): PyVista on 8
# logical CPU processors, ~60 s for 10M rays against ~30k triangles; the
# CUDA LBVH on a GTX Titan X, 0.463 s (v2.1) and 0.228 s with sorted rays
# (v2.2, sort excluded) for 10M rays against 29,284 triangles.
PAPER_CONTEXT = {
    "pyvista_cpu_s_10M_rays_30k_tris": 60.6,
    "titan_x_v2_1_s_10M_rays_29284_tris": 0.463,
    "titan_x_v2_2_sorted_rays_s": 0.228,
}

QUERY_SOURCES = ("paper_2209_02878_amd/csrc/query.hip", "paper_2209_02878_amd/csrc/rsi_device.h",
                 "paper_2209_02878_amd/csrc/rsi_host.h")
TRAFFIC_PROFILE = "profiles/hbm_traffic_k_query_heightfield29768_10Mseg.md"
L2_PROFILE = "profiles/l2_hit_rate_heightfield29768_10Mseg.md"


def query_sources_hash():
    import hashlib
    h = hashlib.sha256()
    for f in QUERY_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def _profile_record(path, tag):
    """key=value pairs of the `tag:` line of a committed profile summary, or
    None when it is missing or was taken from other query sources."""
    import re
    try:
        with open(os.path.join(ROOT, path)) as f:
            text = f.read()
    except OSError:
        return None
    m = re.search(rf"^{tag}: (.*)$", text, re.M)
    if not m:
        return None
    rec = dict(kv.split("=", 1) for kv in m.group(1).split())
    if rec.get("sources") != query_sources_hash():
        return None
    return rec


def measured_traffic():
    """HBM bytes per boolean-query launch from the committed counter runs
    (FETCH_SIZE and WRITE_SIZE, each scaled by a copy of known size)."""
    rec = _profile_record(TRAFFIC_PROFILE, "traffic-record")
    if rec is None:
        return None
    return (float(rec["fetch_kib"]) * float(rec["fetch_scale"]) +
            float(rec["write_kib"]) * float(rec["write_scale"])) * 1024.0


def measured_l2():
    """L2 hit rates (TCC_HIT / (TCC_HIT + TCC_MISS)) per query kernel from the
    committed counter run."""
    rec = _profile_record(L2_PROFILE, "l2-record")
    if rec is None:
        return None
    return {k: float(v) for k, v in rec.items() if k != "sources"}


def cpu_model():
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    import platform
    return platform.processor() or platform.machine()


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def degenerate_fraction(w, n_pick, seed):
    """Near-degenerate segments (the oracle's classifier, delta = 1e-6 of the
    mesh diagonal) in a seeded sample of a workload."""
    import oracle
    idx = np.arange(w.n_r) if n_pick >= w.n_r else np.sort(
        np.random.default_rng(seed).choice(w.n_r, n_pick, replace=False))
    L = float(np.linalg.norm(w.V.astype(np.float64).max(0) - w.V.astype(np.float64).min(0)))
    d = oracle.degenerate(w.V, w.T, w.S[idx], w.E[idx], 1e-6 * L)
    n = int((d != 0).sum())
    return {"sample": int(idx.size), "near_degenerate": n, "fraction": round(n / idx.size, 6)}


EXTRA_SECTIONS = ("c1", "c2var", "c3", "c4", "c5")


def extra_workloads(torch, rsi, wl, dev, time_events, w2, V2, T2, S2, E2, sections=EXTRA_SECTIONS):
    """The other configurations, reported beside the headline: c1 the
    1,922-triangle heightfield; c2var the headline workload on the binary walk
    and with Morton-ordered segments; c3 the 499,280-triangle closed sphere
    (all hits + first hit, boolean, inside test); c4 the differentiable first
    hit on 199,712 triangles; c5 the 64-mesh batch."""
    out = {}
    med = lambda xs: float(np.median(xs))

    if "c1" in sections:
        # the 1,922-triangle heightfield, 100k segments, boolean
        w = wl.config1()
        V, T, S, E = (torch.from_numpy(x).to(dev) for x in (w.V, w.T, w.S, w.E))
        m = rsi.Mesh(V, T)
        o = m.alloc_outputs(w.n_r, "bool")
        q = time_events(lambda: m.query_into(S, E, "bool", o), 20)
        out["heightfield_1922tri_100kseg_bool"] = {"query_ms": round(med(q), 4),
                                                   "msegments_per_s": round(w.n_r / med(q) / 1e3, 2)}
        log(f"1,922-triangle heightfield: bool {med(q):.4f} ms")
        m.close()

    if "c2var" in sections:
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

    if "c3" in sections:
        # closed 499,280-triangle sphere: all crossings (capacity 4) + first hit
        t0 = time.time()
        w = wl.config3()
        log(f"workload {w.name} generated in {time.time() - t0:.1f}s")
        V, T, S, E = (torch.from_numpy(x).to(dev) for x in (w.V, w.T, w.S, w.E))
        m = rsi.Mesh(V, T)
        o = m.alloc_outputs(w.n_r, "all|first", capacity=4)
        b = time_events(lambda: m.rebuild(V, T), 5)
        q = time_events(lambda: m.query_into(S, E, "all|first", o, capacity=4), 5)
        st = m.stats()
        ob = m.alloc_outputs(w.n_r, "bool")
        qb = time_events(lambda: m.query_into(S, E, "bool", ob), 5)
        out["sphere_499280tri_10Mseg_all_first_k4"] = {
            "build_ms": round(med(b), 4), "query_ms": round(med(q), 4),
            "msegments_per_s": round(w.n_r / med(q) / 1e3, 2), "query_bool_ms": round(med(qb), 4),
            "overflowed_segments": int(st["overflow_segments"]), "spilled_crossings": int(st["overflow_crossings"]),
            "deep_pass_segments": int(st["deep_segments"])}
        log(f"sphere all|first: query {med(q):.3f} ms, bool {med(qb):.3f} ms, build {med(b):.3f} ms, stats {st}")
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
        del V, T, S, E, o, ob, P, ins, cnt, ends

    if "c4" in sections:
        # differentiable first hit: 199,712-triangle heightfield, 4M segments
        w = wl.config4()
        Vg, _ = wl.config4_target()
        V, T, S, E = (torch.from_numpy(x).to(dev) for x in (w.V, w.T, w.S, w.E))
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

        def adjoint_call():
            # the library's backward alone (the autograd step adds torch's loss
            # gradient and buffer set-up around it)
            with torch.no_grad():
                _, _, P, tri = rsi.FirstHit.apply(Vp, S, E, m)
                g_p = torch.zeros_like(P)
                g_p[:, 2] = 2 * (P[:, 2] - target)
            torch.cuda.synchronize()
            return time_events(lambda: rsi.rsi_first_hit_backward(m.handle, Vp.detach(), S, E, tri, None, None, g_p),
                               10)

        def adjoint_roofline(times):
            t_ms = med(times)
            # algorithmic traffic per segment: S, E (24 B), triangle id (4 B) and
            # upstream dL/dP (12 B) in, dS and dE (24 B) out, plus t and (u, v)
            # gradients when given (12 B): 76 B
            return {"library_backward_ms": round(t_ms, 4),
                    "hbm_frac_of_76B_per_segment": round(76.0 * w.n_r / (t_ms / 1e3) / 1e9 / PEAK_HBM_GBS, 5)}

        adj = adjoint_roofline(adjoint_call())
        rec = {
            "forward_ms": round(med(f), 4), "forward_backward_ms": round(med(fb), 4),
            "backward_ms": round(med(fb) - med(f), 4),
            "forward_msegments_per_s": round(w.n_r / med(f) / 1e3, 2),
            "forward_backward_msegments_per_s": round(w.n_r / med(fb) / 1e3, 2),
            "fwd_bwd_over_fwd_time": round(med(fb) / med(f), 3), "adjoint": adj}
        log(f"diff first hit: fwd {med(f):.3f} ms, fwd+bwd {med(fb):.3f} ms, adjoint {adj}")
        # the same training step with the segments put in Morton order once
        # (a training loop's segments do not change between steps): the
        # loss is a sum over segments, so its value and dL/dV are those
        # of the input order
        oc = time_events(lambda: m.segment_order(S, E), 3)
        order, So, Eo = m.segment_order(S, E)
        target_in = target
        target = target_in[order.long()].contiguous()
        S_in, E_in = S, E
        S, E = So, Eo
        fo = time_events(fwd, 10)
        fbo = time_events(fwd_bwd, 10)
        adj_o = adjoint_roofline(adjoint_call())
        S, E, target = S_in, E_in, target_in
        rec["morton_ordered_segments"] = {
            "order_once_ms": round(med(oc), 4), "forward_ms": round(med(fo), 4),
            "forward_backward_ms": round(med(fbo), 4), "backward_ms": round(med(fbo) - med(fo), 4),
            "forward_backward_msegments_per_s": round(w.n_r / med(fbo) / 1e3, 2),
            "fwd_bwd_over_fwd_time": round(med(fbo) / med(fo), 3), "adjoint": adj_o}
        log(f"diff first hit, Morton-ordered segments: fwd {med(fo):.3f} ms, fwd+bwd {med(fbo):.3f} ms "
            f"(order once {med(oc):.3f} ms)")
        out["heightfield_199712tri_4Mseg_first_hit_grad"] = rec
        m.close()
        del V, T, S, E, Vp

    if "c5" in sections:
        # 64 meshes: one captured graph (rebuild all + one batched query) per mode,
        # with options chosen by the autotuner on this batch, against 64
        # sequential plain calls (rebuild + query per mesh)
        from paper_2209_02878_amd import tune
        t0 = time.time()
        ws = wl.config5()
        log(f"64-mesh batch generated in {time.time() - t0:.1f}s: {sum(x.n_t for x in ws)} triangles, "
            f"{sum(x.n_r for x in ws)} segments")
        meshes = [(torch.from_numpy(x.V).to(dev), torch.from_numpy(x.T).to(dev)) for x in ws]
        segs = [(torch.from_numpy(x.S).to(dev), torch.from_numpy(x.E).to(dev)) for x in ws]
        singles = [rsi.Mesh(Vm, Tm) for Vm, Tm in meshes]
        ntot = sum(x.n_r for x in ws)
        bt = rsi.Batch(meshes)
        for mode in ("bool", "first"):
            t0 = time.time()
            opts = tune.autotune(bt, segs, mode=mode, kind="batch64", n_t=sum(x.n_t for x in ws), n_r=ntot,
                                 cache_path=None)
            t_tune = time.time() - t0
            for sm in singles:
                sm.set_opts(**opts)  # a new leaf size applies at the rebuild of each sequential step
            souts = [sm.alloc_outputs(Sm.shape[0], mode) for sm, (Sm, _) in zip(singles, segs)]

            def sequential():
                for sm, (Vm, Tm), (Sm, Em), so in zip(singles, meshes, segs, souts):
                    sm.rebuild(Vm, Tm)
                    sm.query_into(Sm, Em, mode, so)

            bouts = bt.alloc_outputs(segs, mode)
            bt.capture(segs, mode, bouts, rebuild=True)
            seq = time_events(sequential, 3)
            rep = time_events(bt.replay, 10)
            torch.cuda.synchronize()
            same = all(torch.equal(bo[key], so[key]) for bo, so in zip(bouts, souts) for key in so)
            out[f"batch_64_meshes_{mode}"] = {
                "n_t": int(sum(x.n_t for x in ws)), "n_r": int(ntot), "tuned_options": opts,
                "autotune_s": round(t_tune, 2),
                "graph_replay_ms": round(med(rep), 4), "sequential_64_calls_ms": round(med(seq), 4),
                "graph_msegments_per_s": round(ntot / med(rep) / 1e3, 2),
                "speedup_vs_sequential": round(med(seq) / med(rep), 3), "identical_to_sequential": bool(same)}
            log(f"batch {mode}: tuned {opts} in {t_tune:.1f}s; graph {med(rep):.3f} ms vs sequential "
                f"{med(seq):.3f} ms, identical={same}")
            del bouts, souts
        bt.close()
        for sm in singles:
            sm.close()
    return out


def cpu_baseline(w, threads_probe, seconds, log):
    """The FP64 oracle (test infrastructure) on a bounded prefix of the
    headline workload, on the host's cores; plus the 1,922-triangle workload
    in full with all threads and with one."""
    import oracle
    from paper_2209_02878_amd import workloads as wl
    threads = oracle.max_threads()
    probe = 100_000
    t1 = time.perf_counter()
    oracle.query(w.V, w.T, w.S[:probe], w.E[:probe])
    dt = time.perf_counter() - t1
    n_s = int(min(w.n_r, max(probe, probe * seconds / max(dt, 1e-6))))
    t1 = time.perf_counter()
    oracle.query(w.V, w.T, w.S[:n_s], w.E[:n_s])
    dt = time.perf_counter() - t1
    rate = n_s / dt
    w1 = wl.config1()
    t1 = time.perf_counter()
    oracle.query(w1.V, w1.T, w1.S, w1.E)
    c1_all = time.perf_counter() - t1
    t1 = time.perf_counter()
    oracle.query(w1.V, w1.T, w1.S, w1.E, threads=1)
    c1_one = time.perf_counter() - t1
    return {
        "value": round(rate / 1e6, 5),
        "unit": "Msegments/s",
        "cores": threads,
        "kind": "oracle",
        "sample": f"first {n_s} of the 10M segments against all 29,768 triangles, FP64 brute force "
                  f"over every pair (box-overlap check, then the exact test), {dt:.1f} s",
        "cpu_model": cpu_model(),
        "pair_tests_per_s": round(n_s * w.n_t / dt, 1),
        "extrapolated_full_10M_s": round(w.n_r / rate, 2),
        "heightfield_1922tri_100kseg_full": {"threads": threads, "s": round(c1_all, 3), "one_thread_s": round(c1_one, 3),
                                             "pair_tests_per_s_one_thread": round(w1.n_r * w1.n_t / c1_one, 1)},
        "paper_context": PAPER_CONTEXT,
    }


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
    ap.add_argument("--extra", default=None,
                    help="comma list of the other workloads to run: " + ", ".join(EXTRA_SECTIONS) +
                         " (with --headline-only: none unless given)")
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

    # ---- the query launches, timed with HIP events on the launch stream
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
    st_all = mesh.stats()
    b_only = time_events(lambda: mesh.rebuild(V, T), reps)
    kb = float(np.mean(q_bool))
    log(f"bool query: mean {kb:.3f} ms, median {np.median(q_bool):.3f} ms; "
        f"all-hits query: median {np.median(q_all):.3f} ms ({st_all}); rebuild: median {np.median(b_only):.3f} ms")

    # ---- algorithmic work of that launch, from the counting variant (untimed)
    mesh.set_counting(True)
    mesh.query_into(S, E, "bool", out_b)
    torch.cuda.synchronize()
    cnt = mesh.counters()
    st_bool = mesh.stats()
    mesh.set_counting(False)
    flops = OPS_PER_BOX_TEST * cnt["box_tests"] + OPS_PER_TRI_TEST * cnt["tri_tests"]
    achieved = flops / (kb / 1e3) / 1e12
    hits = int(out_b["hit"].sum().item())
    lane_visit_share = cnt["node_visits"] / max(1, 64 * cnt["wave_node_steps"])
    log(f"counters: {cnt}; hit fraction {hits / w.n_r:.4f}; lane-visit share {lane_visit_share:.3f}")

    # the FP32 roofline of the other query modes on the same workload: the
    # counting variant gives the tests of each launch, HIP events its time
    out_f = mesh.alloc_outputs(w.n_r, "first")
    q_first = time_events(lambda: mesh.query_into(S, E, "first", out_f), max(5, reps // 2))
    mode_rooflines = {}
    for name, mode, o, times in (("all_hits_k4", "all", out_a, q_all), ("first_hit", "first", out_f, q_first)):
        mesh.set_counting(True)
        mesh.query_into(S, E, mode, o, capacity=4)
        torch.cuda.synchronize()
        c = mesh.counters()
        mesh.set_counting(False)
        ops = OPS_PER_BOX_TEST * c["box_tests"] + OPS_PER_TRI_TEST * c["tri_tests"]
        t_ms = float(np.median(times))
        mode_rooflines[name] = {
            "query_ms": round(t_ms, 4), "fp32_ops_per_launch": int(ops),
            "achieved_tflops": round(ops / (t_ms / 1e3) / 1e12, 4),
            "frac": round(ops / (t_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS, 5),
            "frac_of_unpacked_fp32_78p6": round(ops / (t_ms / 1e3) / 1e12 / PEAK_FP32_TFLOPS_UNPACKED, 5),
            "node_visits_per_segment": round(c["node_visits"] / w.n_r, 4),
            "lane_visit_share": round(c["node_visits"] / max(1, 64 * c["wave_node_steps"]), 4)}
    del out_f
    log(f"other modes: {mode_rooflines}")

    traffic = measured_traffic()
    traffic = None if traffic is None else round(traffic)
    l2 = measured_l2()
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
        "all_hits_over_bool_time": round(float(np.median(q_all) / np.median(q_bool)), 3),
        "all_hits_overflowed_segments": int(st_all["overflow_segments"]),
        "deep_pass_segments_bool": int(st_bool["deep_segments"]),
        "rebuild_ms": round(float(np.median(b_only)), 4),
        "query_first_hit_ms": mode_rooflines["first_hit"]["query_ms"],
        "mode_rooflines": mode_rooflines,
        "hit_fraction": round(hits / w.n_r, 5),
        "work_per_segment": {"node_visits": cnt["node_visits"] / w.n_r, "box_tests": cnt["box_tests"] / w.n_r,
                             "tri_tests": cnt["tri_tests"] / w.n_r},
        "lane_visit_share": round(lane_visit_share, 4),
        "roofline": {
            "bound": "alu",
            "kernel": "k_query<bool> (quantised four-way walk)",
            "achieved": round(achieved, 4),
            "peak": PEAK_FP32_TFLOPS,
            "unit": "TFLOP/s",
            "frac": round(achieved / PEAK_FP32_TFLOPS, 5),
            "frac_of_unpacked_fp32_78p6": round(achieved / PEAK_FP32_TFLOPS_UNPACKED, 5),
            "traffic": traffic,
            "traffic_unit": "HBM bytes per launch (rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated)",
            "hbm_frac": None if traffic is None else round(traffic / (kb / 1e3) / 1e9 / PEAK_HBM_GBS, 5),
            "l2_hit_rate": l2,
            "fp32_ops_per_launch": int(flops),
            "box_tests": int(cnt["box_tests"]), "tri_tests": int(cnt["tri_tests"]),
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

    if args.extra is None:
        sections = [] if args.headline_only else list(EXTRA_SECTIONS)
    else:
        sections = [x for x in args.extra.split(",") if x]
    unknown = set(sections) - set(EXTRA_SECTIONS)
    if unknown:
        raise SystemExit(f"unknown --extra sections: {sorted(unknown)}")
    if sections:
        mesh.close()
        rec["extra"] = extra_workloads(torch, rsi, wl, dev, time_events, w, V, T, S, E, set(sections))

    if not args.no_cpu_baseline:
        # near-degenerate segments per workload (oracle classifier on samples)
        t0 = time.time()
        rec["near_degenerate"] = {
            "heightfield_1922tri_100kseg": degenerate_fraction(wl.config1(), 100_000, 1),
            "heightfield_29768tri_10Mseg": degenerate_fraction(w, 50_000, 2),
            # (4,000 and 50,000 segments drawn by the same recipes as the full workloads)
            "sphere_499280tri_10Mseg": degenerate_fraction(wl.config3(n_r=4_000), 4_000, 3),
            "heightfield_199712tri_4Mseg": degenerate_fraction(wl.config4(n_r=50_000), 50_000, 4),
        }
        log(f"near-degenerate samples ({time.time() - t0:.1f}s): {rec['near_degenerate']}")
        rec["cpu_baseline"] = cpu_baseline(w, None, args.cpu_seconds, log)
        log(f"cpu baseline: {rec['cpu_baseline']}")
    if not sections:
        mesh.close()
    print(json.dumps(rec), flush=True)


if __name__ == "__main__":
    main()
