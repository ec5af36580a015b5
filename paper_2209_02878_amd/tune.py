"""Autotuning of the query launch options, with a JSON cache.

The timing itself runs in the library (`rsi_tune`: each candidate option set
is applied, warmed up and timed with HIP events; the fastest stays applied).
This module chooses the candidates -- a staged search over the options that
matter most first -- and remembers the winner per (device, workload kind,
mode, size bucket) in a JSON file, so a later run of the same shape can skip
the search.

Tunable: branching (the binary tree or its four-way view), block size, LDS
stack depth, leaf size (needs a rebuild), defer and refill lane thresholds.
"""
from __future__ import annotations

import json
import math
import os

from . import rsi

DEFAULT_CACHE = os.environ.get("RSI_TUNE_CACHE", os.path.join(os.path.expanduser("~"), ".cache", "rsi_tune.json"))

# staged search: each stage varies some options on top of the best so far
STAGES = [
    [{"branching": w, "block_size": b} for w in (2, 4) for b in (64, 128, 256)],
    # LDS stack entries per lane of the main pass (deeper walks go to the deep pass)
    [{"stack_depth": s} for s in (8, 12, 16, 20, 24, 32)],
    [{"defer_lanes": d, "refill_lanes": r} for d in (16, 32, 48) for r in (16, 24, 32, 48)],
    [{"leaf_size": leaf} for leaf in (1, 2, 4)],
]


def size_bucket(n: int) -> int:
    """Power-of-two bucket of a size (sizes within a factor ~1.4 share one)."""
    return int(round(math.log2(max(int(n), 1))))


def cache_key(device: str, kind: str, mode, n_t: int, n_r: int) -> str:
    return f"{device}|{kind}|{rsi.parse_mode(mode)}|t{size_bucket(n_t)}|r{size_bucket(n_r)}"


def load_cache(path: str = DEFAULT_CACHE) -> dict:
    try:
        with open(path) as f:
            data = json.load(f)
        return data if isinstance(data, dict) else {}
    except (OSError, ValueError):
        return {}


def save_cache(cache: dict, path: str = DEFAULT_CACHE) -> None:
    d = os.path.dirname(path)
    if d:
        os.makedirs(d, exist_ok=True)
    tmp = f"{path}.tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(cache, f, indent=1, sort_keys=True)
    os.replace(tmp, path)


def device_name() -> str:
    import torch
    p = torch.cuda.get_device_properties(torch.cuda.current_device())
    return getattr(p, "gcnArchName", None) or p.name


def staged_search(run_stage, base: dict | None = None) -> tuple[dict, list]:
    """run_stage(candidates) -> (best index, times); returns the best option
    dict and the log of (candidate, ms)."""
    best = dict(base or {})
    log = []
    for stage in STAGES:
        cands = [{**best, **c} for c in stage]
        i, ms = run_stage(cands)
        log.extend(zip(cands, ms))
        best = cands[i]
    return best, log


def autotune(target, *args, mode="bool", kind="mesh", n_t=0, n_r=0, cache_path: str | None = DEFAULT_CACHE,
             reps: int = 3) -> dict:
    """Tune `target` (an rsi.Mesh with args (S, E) or an rsi.Batch with args
    (segments,)) unless the cache already holds options for this shape; the
    chosen options are applied to the target and returned."""
    key = cache_key(device_name(), kind, mode, n_t, n_r)
    cache = load_cache(cache_path) if cache_path else {}
    if key in cache:
        opts = cache[key]["opts"]
        # a one-candidate run applies the options (rebuilding for a new leaf size)
        target.tune(*args, mode, [opts], reps=1)
        return opts
    best, log = staged_search(lambda c: target.tune(*args, mode, c, reps=reps))
    if cache_path:
        cache[key] = {"opts": best, "ms": min(ms for _, ms in log)}
        save_cache(cache, cache_path)
    return best
