"""Host logic of bench.py (no GPU): the traffic summary lookup, the tile
height recovered from a launch's grid size, and the one-GPU guard."""
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _launch_threads(n, rows, strip):
    """Threads of one launch: 4-wave blocks, rounded up to 8 blocks (one per XCD)."""
    tiles = -(-n // strip) * -(-n // rows)
    blocks = -(-tiles // 4)
    return -(-blocks // 8) * 8 * 256


@pytest.mark.parametrize("rows", [1, 4, 12, 15, 19, 25, 64])
def test_rows_from_grid_inverts_the_launch_shape(rows):
    for strip in (56, 60):
        got = bench.rows_from_grid(_launch_threads(2048, rows, strip), 2048, strip)
        # the smallest height with the same launch shape
        assert got is not None and got <= rows
        assert _launch_threads(2048, got, strip) == _launch_threads(2048, rows, strip)


def _summary(tmp_path, monkeypatch, **extra):
    s = {"kernel_source_sha256": bench.kernel_source_hash(), "grid": 2048, "tile_rows": 12,
         "stage": {"fused": {"bytes": 700, "tile_rows": 12}}, "bytes_per_launch": 900,
         "fused_by_rows": {"15": {"bytes": 750}, "19": {"bytes": 760}}}
    s.update(extra)
    path = tmp_path / "traffic.json"
    path.write_text(json.dumps(s))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(path))


def test_traffic_lookup_by_height(tmp_path, monkeypatch):
    _summary(tmp_path, monkeypatch)
    assert bench.load_traffic(2048, "fp32", "superbee", 15, fused=True) == (750, 15)
    assert bench.load_traffic(2048, "fp32", "superbee", 19, fused=True) == (760, 19)
    # a fused height the passes did not cover: the profiled entry, with its height
    assert bench.load_traffic(2048, "fp32", "superbee", 13, fused=True) == (700, 12)
    # unfused: only at the profiled height
    assert bench.load_traffic(2048, "fp32", "superbee", 12) == (900, 12)
    assert bench.load_traffic(2048, "fp32", "superbee", 16) is None
    # other workloads have no summary
    assert bench.load_traffic(4096, "fp32", "superbee", 12) is None
    assert bench.load_traffic(2048, "fp64", "superbee", 12) is None
    assert bench.load_traffic(2048, "fp32", "mc", 12) is None


def test_traffic_ignored_once_the_kernels_change(tmp_path, monkeypatch):
    _summary(tmp_path, monkeypatch, kernel_source_sha256="0" * 64)
    assert bench.load_traffic(2048, "fp32", "superbee", 12) is None
    assert bench.load_traffic(2048, "fp32", "superbee", 15, fused=True) is None


def test_committed_traffic_summary_is_well_formed():
    # (bench.py reports it only while its source hash matches the kernels)
    with open(bench.TRAFFIC_FILE) as fh:
        t = json.load(fh)
    assert len(t["kernel_source_sha256"]) == 64
    assert t["grid"] == 2048 and t["bytes_per_launch"] > 0 and t["fused_by_rows"]
    assert 1.9 < t["fetch_factor"] < 2.1 and 0.9 < t["write_factor"] < 1.1


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
