"""File formats and arguments of the command line (paper Sections 2.3-2.5), on the CPU."""
import numpy as np
import pytest

from paper_2209_02878_amd import cli


def test_input_files_round_trip(tmp_path):
    rng = np.random.default_rng(0)
    V = rng.normal(size=(10, 3)).astype(np.float32)
    T = rng.integers(0, 10, (7, 3)).astype(np.int32)
    S = rng.normal(size=(5, 3)).astype(np.float32)
    E = rng.normal(size=(5, 3)).astype(np.float32)
    cli.write_inputs(str(tmp_path), V, T, S, E)
    # little-endian packed arrays, 3 values per record
    raw = (tmp_path / "triangles_i32").read_bytes()
    assert raw == T.astype("<i4").tobytes()
    got = cli.read_inputs(*[str(tmp_path / n) for n in cli.DEFAULT_NAMES])
    for a, b in zip(got, (V, T, S, E)):
        assert a.dtype == b.dtype and np.array_equal(a, b)


def test_input_validation(tmp_path):
    np.arange(4, dtype="<f4").tofile(tmp_path / "bad")
    np.zeros(6, "<f4").tofile(tmp_path / "v")
    np.zeros(3, "<i4").tofile(tmp_path / "t")
    with pytest.raises(ValueError):
        cli.read_inputs(str(tmp_path / "bad"), str(tmp_path / "t"), str(tmp_path / "v"), str(tmp_path / "v"))
    np.zeros(9, "<f4").tofile(tmp_path / "s3")
    with pytest.raises(ValueError):
        cli.read_inputs(str(tmp_path / "v"), str(tmp_path / "t"), str(tmp_path / "v"), str(tmp_path / "s3"))


def test_argument_forms():
    p, silent, mode, out = cli.parse_args([])
    assert p[0].endswith("vertices_f32") and not silent and mode == "default"
    p, silent, mode, out = cli.parse_args(["a", "b", "c", "d", "silent"])
    assert p == ["a", "b", "c", "d"] and silent and mode == "default"
    p, silent, mode, out = cli.parse_args(["a", "b", "c", "d", "default", "barycentric", "--out", "x"])
    assert not silent and mode == "barycentric" and out == "x"
    with pytest.raises(SystemExit):
        cli.parse_args(["a", "b"])
    with pytest.raises(SystemExit):
        cli.parse_args(["a", "b", "c", "d", "default", "nonsense"])


def test_output_files(tmp_path):
    res = {"intersecting_rays": np.array([1, 4], np.int32), "distances": np.array([0.5, 2.0], np.float32)}
    paths = cli.write_outputs(str(tmp_path), res)
    assert sorted(p.split("/")[-1] for p in paths) == ["distances_f32", "intersecting_rays_i32"]
    assert np.array_equal(np.fromfile(tmp_path / "distances_f32", "<f4"), res["distances"])
