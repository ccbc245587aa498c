"""Host logic of bench.py: which committed counter summary applies to a bench line."""

import hashlib
import json
import os

import bench


def _tree(tmp_path, src=b"kernel source"):
    csrc = tmp_path / "paper_1612_04846_amd" / "csrc"
    csrc.mkdir(parents=True)
    (csrc / "bura_kernels.hip").write_bytes(src)
    (tmp_path / "profiles").mkdir()
    return hashlib.sha256(src).hexdigest()[:16]


def _summary(tmp_path, name, sha, kclass, tiles, kernel_tile, traffic, workload="w2d"):
    lines = ["# HBM traffic counters", "", "- a bullet: not a key", "",
             f"traffic_bytes_per_launch: {traffic}", f"kernel_source_sha256_prefix: {sha}",
             f"kernel_class: {kclass}", f"workload: {workload}", f"tiles: {json.dumps(tiles)}"]
    if kernel_tile is not None:
        lines.append(f"kernel_tile: {kernel_tile}")
    (tmp_path / "profiles" / name).write_text("\n".join(lines) + "\n")


def test_counter_summary_matches_on_the_kernels_own_launch_shape(tmp_path, monkeypatch):
    sha = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "spmv_hbm_counters.md", sha, "spmv", [[0, 0, 0, 0, 0]], 0, 111)
    _summary(tmp_path, "up_hbm_counters.md", sha, "up_fine", [[0, 0, 0, 0, 0]], 0, 222)
    # another level's or another kernel's shape does not matter
    assert bench.counter_traffic("w2d", "spmv", [[0, 1, 2, 1, 2]]) == 111
    assert bench.counter_traffic("w2d", "up_fine", [[2, 1, 0, 2, 2]]) == 222
    # the kernel's own shape does
    assert bench.counter_traffic("w2d", "spmv", [[2, 0, 0, 0, 0]]) is None
    assert bench.counter_traffic("w2d", "up_fine", [[0, 0, 1, 0, 0]]) is None
    # several plans: every one must use the summary's shape
    assert bench.counter_traffic("w2d", "spmv", [[0, 0, 0], [0, 2, 2]]) == 111
    assert bench.counter_traffic("w2d", "spmv", [[0, 0, 0], [1, 0, 0]]) is None
    # other workload or kernel class
    assert bench.counter_traffic("other", "spmv", [[0, 0, 0]]) is None
    assert bench.counter_traffic("w2d", "down_fine", [[0, 0, 0]]) is None


def test_counter_summary_of_other_kernel_source_is_ignored(tmp_path, monkeypatch):
    _tree(tmp_path, b"new source")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    old = hashlib.sha256(b"old source").hexdigest()[:16]
    _summary(tmp_path, "spmv_hbm_counters.md", old, "spmv", [[0, 0, 0]], 0, 111)
    assert bench.counter_traffic("w2d", "spmv", [[0, 0, 0]]) is None


def test_classes_without_shape_variants_need_the_same_tiles(tmp_path, monkeypatch):
    sha = _tree(tmp_path)
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    _summary(tmp_path, "smooth_hbm_counters.md", sha, "smooth_fine", [], None, 333, workload="w3d")
    assert bench.counter_traffic("w3d", "smooth_fine", []) == 333
    assert bench.counter_traffic("w3d", "smooth_fine", [[0]]) is None
    assert "smooth_fine" not in bench.TILE_INDEX
    assert os.path.basename(bench.__file__) == "bench.py"
