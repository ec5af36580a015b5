"""Host logic of the autotuner: size buckets, cache keys, the JSON cache and
the staged search (no device needed)."""
from paper_2209_02878_amd import tune


def test_size_bucket_and_key():
    assert tune.size_bucket(1) == 0
    assert tune.size_bucket(1024) == 10
    assert tune.size_bucket(29_768) == tune.size_bucket(30_000)
    assert tune.size_bucket(10_000_000) == 23
    k = tune.cache_key("gfx950", "mesh", "bool", 29_768, 10_000_000)
    assert k == "gfx950|mesh|1|t15|r23"
    assert tune.cache_key("gfx950", "mesh", "first|bool", 1, 1).split("|")[2] == "3"


def test_cache_round_trip(tmp_path):
    p = str(tmp_path / "sub" / "cache.json")
    assert tune.load_cache(p) == {}
    tune.save_cache({"a": {"opts": {"block_size": 64}, "ms": 1.5}}, p)
    assert tune.load_cache(p) == {"a": {"opts": {"block_size": 64}, "ms": 1.5}}
    with open(p, "w") as f:
        f.write("not json")
    assert tune.load_cache(p) == {}


def test_staged_search_keeps_best_of_each_stage():
    seen = []

    def run_stage(cands):
        seen.append(cands)
        # prefer branching 4 / block 64, stack 12, then defer 48 refill 16, then leaf 2
        def cost(c):
            return (abs(c.get("branching", 2) - 4) + abs(c.get("block_size", 128) - 64)
                    + abs(c.get("stack_depth", 0) - 12)
                    + abs(c.get("defer_lanes", 32) - 48) + abs(c.get("refill_lanes", 32) - 16)
                    + abs(c.get("leaf_size", 1) - 2))
        ms = [float(cost(c)) for c in cands]
        return ms.index(min(ms)), ms

    best, log = tune.staged_search(run_stage)
    assert best == {"branching": 4, "block_size": 64, "stack_depth": 12, "defer_lanes": 48, "refill_lanes": 16,
                    "leaf_size": 2}
    assert len(seen) == len(tune.STAGES)
    # later stages carry the earlier winners
    assert all(c["block_size"] == 64 for c in seen[1])
    assert len(log) == sum(len(s) for s in tune.STAGES)
