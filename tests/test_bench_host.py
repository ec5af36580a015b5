"""Host logic of the benchmark (no GPU): the profile records it reads are
used only while the query sources hash to the value they were taken with,
and a run on more than one GPU is refused before anything is measured."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_profile_record_follows_the_sources(tmp_path, monkeypatch):
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "query_sources_hash", lambda: "abc123")
    (tmp_path / "p.md").write_text("text\n\ntraffic-record: kernel=k sources=abc123 fetch_kib=10.5 write_kib=2.0 "
                                   "fetch_scale=2.0 write_scale=1.0\n")
    rec = bench._profile_record("p.md", "traffic-record")
    assert rec == {"kernel": "k", "sources": "abc123", "fetch_kib": "10.5", "write_kib": "2.0",
                   "fetch_scale": "2.0", "write_scale": "1.0"}
    # taken from other sources: not used
    (tmp_path / "q.md").write_text("traffic-record: kernel=k sources=ffff fetch_kib=1 write_kib=1 "
                                   "fetch_scale=1 write_scale=1\n")
    assert bench._profile_record("q.md", "traffic-record") is None
    # missing file or line
    assert bench._profile_record("none.md", "traffic-record") is None
    assert bench._profile_record("p.md", "l2-record") is None


def test_measured_traffic_scales_the_counters(monkeypatch):
    monkeypatch.setattr(bench, "_profile_record", lambda path, tag: {
        "sources": "x", "fetch_kib": "100", "write_kib": "50", "fetch_scale": "2.0", "write_scale": "1.0"})
    assert bench.measured_traffic() == (100 * 2.0 + 50 * 1.0) * 1024.0


def test_sources_hash_covers_the_query_sources():
    h = bench.query_sources_hash()
    assert len(h) == 16 and int(h, 16) >= 0
    for f in bench.QUERY_SOURCES:
        assert os.path.exists(os.path.join(ROOT, f)), f


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "one GPU" in r.stderr
    assert r.stdout.strip() == ""
