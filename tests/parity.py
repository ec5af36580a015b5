"""Comparison of GPU query results with the FP64 oracle (test helper).

Rules (the acceptance bar of the parity tests):
* segments the oracle classifies as near-degenerate (within delta = 1e-6 of
  the mesh's bounding-box diagonal from a triangle edge, an endpoint within
  delta of a triangle, or two crossings within delta of each other) are
  counted and excluded; every other segment must match
* flags, crossing counts, first-hit triangle ids and crossing-list ids:
  bit-exact
* t: |dt| <= 1e-5 (t is already relative to the segment length)
* hit point: max-norm error <= 1e-5 * L; u, v: |d| <= 1e-5
"""
from __future__ import annotations

import numpy as np

import oracle

T_TOL = 1e-5
REL_DELTA = 1e-6


def mesh_extent(V) -> float:
    V = np.asarray(V, np.float64)
    return float(np.linalg.norm(V.max(0) - V.min(0))) if V.size else 1.0


def oracle_reference(V, T, S, E, cap=0, threads=0):
    ref = oracle.query(V, T, S, E, cap=cap, threads=threads)
    L = mesh_extent(V)
    ref["degenerate"] = oracle.degenerate(V, T, S, E, REL_DELTA * L, threads=threads)
    ref["extent"] = L
    return ref


def _np(x):
    return x.detach().cpu().numpy() if hasattr(x, "detach") else np.asarray(x)


def compare(ref, got, modes, cap=0, spill=None):
    """Return a dict of mismatch counts (all zero = parity) and statistics."""
    ok = ref["degenerate"] == 0
    L = ref["extent"]
    rep = {"n": int(ok.size), "degenerate": int((~ok).sum()), "hits": int((ref["count"][ok] > 0).sum())}
    if "bool" in modes:
        h = _np(got["hit"]).astype(bool)
        rep["bool_mismatch"] = int((h[ok] != (ref["count"][ok] > 0)).sum())
    if "first" in modes:
        tri = _np(got["tri"])
        t = _np(got["t"]).astype(np.float64)
        uv = _np(got["uv"]).astype(np.float64)
        P = _np(got["point"]).astype(np.float64)
        rep["first_tri_mismatch"] = int((tri[ok] != ref["first_tri"][ok]).sum())
        hit = ok & (ref["first_tri"] >= 0) & (tri == ref["first_tri"])
        dt = np.abs(t[hit] - ref["first_tuv"][hit, 0])
        duv = np.abs(uv[hit] - ref["first_tuv"][hit, 1:]).max(1) if hit.any() else np.zeros(0)
        dP = np.abs(P[hit] - ref["first_p"][hit]).max(1) if hit.any() else np.zeros(0)
        rep["first_t_bad"] = int((dt > T_TOL).sum())
        rep["first_uv_bad"] = int((duv > T_TOL).sum())
        rep["first_p_bad"] = int((dP > T_TOL * L).sum())
        rep["first_t_maxerr"] = float(dt.max()) if dt.size else 0.0
        miss = ok & (ref["first_tri"] < 0)
        rep["first_miss_bad"] = int((~np.isinf(t[miss])).sum())
    if "all" in modes:
        cnt = _np(got["count"])
        ids = _np(got["ids"])
        ts = _np(got["ts"]).astype(np.float64)
        rep["count_mismatch"] = int((cnt[ok] != ref["count"][ok]).sum())
        k = min(cap, ref["list_tri"].shape[1])
        rc = np.minimum(ref["count"], k)
        bad_ids = bad_t = 0
        for c in range(k):
            m = ok & (rc > c)
            bad_ids += int((ids[m, c] != ref["list_tri"][m, c]).sum())
            same = m & (ids[:, c] == ref["list_tri"][:, c])
            bad_t += int((np.abs(ts[same, c] - ref["list_t"][same, c]) > T_TOL).sum())
            pad = ok & (rc <= c)
            bad_ids += int((ids[pad, c] != -1).sum())
        rep["list_id_mismatch"] = bad_ids
        rep["list_t_bad"] = bad_t
        if spill is not None:
            rep.update(compare_spill(ref, spill, ok))
    return rep


def compare_spill(ref, spill, ok):
    seg = _np(spill["seg"])
    off = _np(spill["offset"])
    cnt = _np(spill["count"])
    ids = _np(spill["ids"])
    ts = _np(spill["ts"]).astype(np.float64)
    full = ref.get("full_lists")
    bad = 0
    checked = 0
    for s, o, c in zip(seg, off, cnt):
        if not ok[s] or full is None:
            continue
        want = full[s]
        checked += 1
        if c != len(want) or list(ids[o:o + c]) != [w[1] for w in want]:
            bad += 1
            continue
        if np.any(np.abs(ts[o:o + c] - np.array([w[0] for w in want])) > T_TOL):
            bad += 1
    return {"spill_segments": int(seg.size), "spill_checked": checked, "spill_bad": bad}


def assert_parity(rep):
    bad = {k: v for k, v in rep.items()
           if (k.endswith("mismatch") or k.endswith("_bad")) and v}
    assert not bad, f"parity failures: {bad}; report: {rep}"
