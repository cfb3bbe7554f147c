"""Host logic of bench.py (no GPU): the counter summary written from
rocprofv3 CSVs and its lookup, the parity records, the coupled-curve
comparison, the host description and the one-GPU guard."""
import csv
import json
import os
import subprocess
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def _csv(path, rows):
    os.makedirs(path, exist_ok=True)
    with open(os.path.join(path, "x_counter_collection.csv"), "w", newline="") as fh:
        w = csv.DictWriter(fh, fieldnames=["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"])
        w.writeheader()
        for r in rows:
            w.writerow(dict(zip(["Kernel_Name", "Grid_Size", "Counter_Name", "Counter_Value"], r)))


def test_profile_summary_calibrates_by_the_copy_kernel(tmp_path, monkeypatch):
    """FETCH_SIZE and WRITE_SIZE are scaled by what they read for a copy of
    known size; SQ counters are averaged per launch."""
    monkeypatch.setattr(bench, "kernel_code_hash", lambda *a, **k: "c" * 64)
    k = "void fdm::(anonymous namespace)::" + bench.HEADLINE_KERNEL + "(fdm::InstDev, long, int, int, int)"
    c = "void fdm::(anonymous namespace)::" + bench.COPY_KERNEL + "(float*, float const*, long)"
    n = 1024                                   # copy of 4 MiB each way = 4096 KiB
    _csv(str(tmp_path / "f"), [(k, 1, "FETCH_SIZE", 1000), (k, 1, "FETCH_SIZE", 1200), (c, 1, "FETCH_SIZE", 2048)])
    _csv(str(tmp_path / "w"), [(k, 1, "WRITE_SIZE", 3000), (c, 1, "WRITE_SIZE", 4096)])
    _csv(str(tmp_path / "s"), [(k, 1, "SQ_INSTS_VALU", 100.0), (k, 1, "SQ_INSTS_VALU", 300.0),
                               (k, 1, "SQ_INSTS_MFMA", 0.0), (k, 1, "SQ_WAVES", 50.0)])
    out = tmp_path / "p.json"
    bench.write_profile_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "s"), str(out), n, 43)
    p = json.loads(out.read_text())
    e = p["by_rows"]["43"]
    assert e["fetch_factor"] == 2.0 and e["write_factor"] == 1.0
    assert e["bytes_per_launch"] == round((1100 * 2.0 + 3000 * 1.0) * 1024)
    assert e["sq_per_launch"] == {"SQ_INSTS_VALU": 200.0, "SQ_INSTS_MFMA": 0.0, "SQ_WAVES": 50.0}
    assert p["kernel_code_sha256"] == "c" * 64
    # a second height joins the first (same sources)
    _csv(str(tmp_path / "f"), [(k, 1, "FETCH_SIZE", 900), (c, 1, "FETCH_SIZE", 2048)])
    bench.write_profile_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "s"), str(out), n, 60)
    p = json.loads(out.read_text())
    assert list(p["by_rows"]) == ["43", "60"]
    assert p["by_rows"]["60"]["bytes_per_launch"] == round((900 * 2.0 + 3000 * 1.0) * 1024)
    # looked up only at a profiled height, and only while the kernels are unchanged
    monkeypatch.setattr(bench, "PROFILE_FILE", str(out))
    assert bench.profiled_heights() == [43, 60]
    assert bench.load_profile(43)["bytes_per_launch"] == round((1100 * 2.0 + 3000 * 1.0) * 1024)
    assert bench.load_profile(42) is None
    p["kernel_code_sha256"] = "0" * 64
    out.write_text(json.dumps(p))
    assert bench.load_profile(43) is None and bench.profiled_heights() == []
    # a summary of other kernel code is replaced, not merged
    bench.write_profile_summary(str(tmp_path / "f"), str(tmp_path / "w"), str(tmp_path / "s"), str(out), n, 50)
    assert list(json.loads(out.read_text())["by_rows"]) == ["50"]


def test_kernel_code_hash_reads_the_built_kernel():
    """The hash covers one kernel's machine code and descriptor in the
    library's gfx950 code object: stable, different per kernel, None for a
    missing kernel or library."""
    if not os.path.exists(bench.LIB_FILE):
        pytest.skip("libfdm.so not built")
    h = bench.kernel_code_hash()
    assert h is not None and len(h) == 64 and h == bench.kernel_code_hash()
    other = bench.HEADLINE_SYMBOL.replace("ILi3ELi0ELb1ELb0E", "ILi2ELi0ELb0ELb0E")
    assert bench.kernel_code_hash(symbol=other) not in (None, h)
    assert bench.kernel_code_hash(symbol="no_such_kernel") is None
    assert bench.kernel_code_hash(path=os.path.join(ROOT, "bench.py")) is None


def test_parity_record_hand_values():
    a = (np.array([[1.0, -1.0]], np.float32), np.array([[2.0, 0.0]], np.float32))    # sum|a| 4, max 2
    o = (np.array([[1.0, -1.0]]), np.array([[1.5, 0.5]]))
    g = (np.array([[1.0, -0.5]]), np.array([[1.5, 0.5]]))
    r = bench.parity_record(g, o, a, 7, 1e-5)
    assert r["rel_l1"] == pytest.approx(0.5 / 4) and r["rel_linf"] == pytest.approx(0.5 / 2)
    # totals: a11 0 -> 0.5 (g), a12 2 -> 2
    assert r["drift"] == pytest.approx(0.5 / 4) and r["oracle_drift"] == 0.0
    assert r["steps"] == 7 and r["bar_rel_l1"] == 1e-5


def test_coupled_curve_parity(tmp_path, monkeypatch):
    ref = [{"step": 100 * (i + 1), "eps13": 0.01 * (i + 1), "sigma13": 0.02 * (i + 1), "phi_mean": -0.01,
            "sum_abs": 10.0} for i in range(3)]
    cols = ["step", "eps13", "sigma13", "phi_mean", "sum_abs"]
    path = tmp_path / "g.json"
    path.write_text(json.dumps({"columns": cols, "history": [[r[c] for c in cols] for r in ref]}))
    monkeypatch.setattr(bench, "GOLDEN_C4", str(path))
    hist = [dict(r) for r in ref]
    hist[1]["sigma13"] += 0.0006                   # over max |sigma13| = 0.06: 1e-2
    hist[2]["sum_abs"] -= 0.2                      # over s0 = 20: 1e-2
    out = bench.coupled_curve_parity({"hist": hist, "s0": 20.0, "steps": 5000})
    assert out["sigma13_max_dev"] == pytest.approx(1e-2) and out["sum_abs_max_dev"] == pytest.approx(1e-2)
    assert out["eps13_max_dev"] == 0.0 and out["records"] == 3
    assert bench.coupled_curve_parity({"hist": hist, "s0": 20.0, "steps": 100}) is None


def test_host_description():
    h = bench.host_description()
    assert h["nproc"] == os.cpu_count() and "cpu_model" in h and "OMP_NUM_THREADS" in h


def test_committed_counter_summary_is_well_formed():
    # (bench.py reports it only while its code hash matches the built kernel)
    if not os.path.exists(bench.PROFILE_FILE):
        pytest.skip("no counter summary committed yet")
    with open(bench.PROFILE_FILE) as fh:
        t = json.load(fh)
    assert len(t["kernel_code_sha256"]) == 64 and t["grid"] == 4096 and t["by_rows"]
    for rows, e in t["by_rows"].items():
        assert int(rows) > 0 and e["bytes_per_launch"] > 0
        assert 1.9 < e["fetch_factor"] < 2.1 and 0.9 < e["write_factor"] < 1.1
        assert e["sq_per_launch"]["SQ_INSTS_VALU"] > 0 and e["sq_per_launch"].get("SQ_INSTS_MFMA", 0) == 0


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
