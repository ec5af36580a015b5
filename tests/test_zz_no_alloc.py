"""rsi_query_noalloc (the query entry point that allocates nothing, for
callers that cannot call hipMalloc) against rsi_query through the C ABI: the
same kernels on the same inputs, so every output must agree bit for bit, on
two calls in a row, the second with fewer segments.  The first call is large
enough to run as two parts of the fixed scratch array; a sample of both is
also held to the FP64 oracle (paper Section 1 problem, Section 3.2 walk)."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")

from paper_2209_02878_amd import rsi
from paper_2209_02878_amd import workloads as wl
from tests import parity

pytestmark = pytest.mark.gpu
DEV = "cuda"


def _t(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a)).to(device=DEV, dtype=dtype).contiguous()


def _oracle_sample(w, S, E, got, idx):
    """First-hit ids and counts of the sampled segments against the oracle,
    on the segments the classifier finds non-degenerate."""
    ref = parity.oracle_reference(w.V, w.T, S[idx], E[idx], cap=1)
    ok = ref["degenerate"] == 0
    assert ok.sum() > 0.9 * idx.size
    cnt = got["count"].cpu().numpy()[idx]
    tri = got["tri"].cpu().numpy()[idx]
    hit = got["hit"].cpu().numpy()[idx]
    assert np.array_equal(cnt[ok], ref["count"][ok])
    assert np.array_equal(tri[ok], ref["first_tri"][ok])
    assert np.array_equal(hit[ok].astype(bool), ref["count"][ok] > 0)
    t = got["t"].cpu().numpy()[idx].astype(np.float64)
    h = ok & (ref["first_tri"] >= 0)
    assert np.all(np.abs(t[h] - ref["first_tuv"][h, 0]) <= 1e-5)


def test_noalloc_query_equals_query_on_two_calls():
    w = wl.config2(n_r=5_000_000)
    V, T = _t(w.V), _t(w.T, torch.int32)
    S, E = _t(w.S), _t(w.E)
    mesh = rsi.Mesh(V, T)
    mode = "bool|first|count"
    rng = np.random.default_rng(7)
    for n in (w.n_r, 300_001):
        print(f"noalloc call: n_r={n} mode={mode}", flush=True)
        Sn, En = S[:n].contiguous(), E[:n].contiguous()
        ref = mesh.query_into(Sn, En, mode, mesh.alloc_outputs(n, mode))
        got = mesh.alloc_outputs(n, mode)
        for v in got.values():
            v.fill_(0x5A) if v.dtype == torch.uint8 else v.fill_(-7)
        mesh.query_noalloc_into(Sn, En, mode, got)
        st = mesh.stats()
        assert st["walk_cut"] == 0 and st["stack_dropped"] == 0
        torch.cuda.synchronize()
        for key in ref:
            assert torch.equal(ref[key], got[key]), key
        idx = np.sort(rng.choice(n, 3000, replace=False))
        _oracle_sample(w, w.S[:n], w.E[:n], got, idx)
    mesh.close()


def test_noalloc_query_edge_cases():
    w = wl.config1(n_r=2_000)
    mesh = rsi.Mesh(_t(w.V), _t(w.T, torch.int32))
    S, E = _t(w.S), _t(w.E)
    out = mesh.alloc_outputs(w.n_r, "bool")
    with pytest.raises(rsi.RsiError, match="RSI_ALL_HITS"):
        mesh.query_noalloc_into(S, E, "all", mesh.alloc_outputs(w.n_r, "all"))
    # n_r = 0 is a no-op
    mesh.query_noalloc_into(S[:0].contiguous(), E[:0].contiguous(), "bool", out)
    ref = mesh.query(S, E, "bool")
    mesh.query_noalloc_into(S, E, "bool", out)
    torch.cuda.synchronize()
    assert torch.equal(out["hit"], ref["hit"])
    mesh.close()
    # an empty mesh: every segment misses
    empty = rsi.Mesh(_t(w.V), torch.zeros((0, 3), dtype=torch.int32, device=DEV))
    o = empty.alloc_outputs(w.n_r, "bool|first")
    empty.query_noalloc_into(S, E, "bool|first", o)
    torch.cuda.synchronize()
    assert int(o["hit"].sum()) == 0 and bool((o["tri"] == -1).all())
    empty.close()
