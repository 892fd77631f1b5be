"""Host-side pieces of bench.py (CPU): the one-GPU guard, the rocprofv3
traffic summary, the kernel-source hash that invalidates it, and the
roofline objects."""
import json
import os
import sqlite3
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def _counter_db(path, counter, rows):
    con = sqlite3.connect(path)
    con.execute("create table counters_collection(dispatch_id int, kernel_name text, "
                "counter_name text, value real)")
    for i, (name, v) in enumerate(rows):
        con.execute("insert into counters_collection values (?, ?, ?, ?)", (i, name, counter, v))
    con.commit()
    con.close()


def test_traffic_summary_scales_by_the_copy(tmp_path, monkeypatch):
    das = "void bf::das_lds_kernel<1, 0, 2, 2>(bf::DasArgs, bf::LdsCfg)"
    # FETCH_SIZE reads half the bytes of the 512 MiB copy, WRITE_SIZE all of them
    _counter_db(tmp_path / "f.db", "FETCH_SIZE",
                [("fill", 0.0), ("copy", 262144.0), (das, 1000.0), (das, 1002.0)])
    _counter_db(tmp_path / "w.db", "WRITE_SIZE",
                [("fill", 524288.0), ("copy", 524288.0), (das, 30.0), (das, 32.0)])
    out = tmp_path / "traffic.json"
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    bench.traffic_summary(str(tmp_path / "f.db"), str(tmp_path / "w.db"))
    t = json.loads(out.read_text())
    assert t["fetch_scale"] == pytest.approx(2.0) and t["write_scale"] == pytest.approx(1.0)
    assert t["fetch_kib_raw"] == pytest.approx(1001.0) and t["write_kib_raw"] == pytest.approx(31.0)
    assert t["das_hbm_bytes_per_launch"] == round((1001.0 * 2 + 31.0) * 1024)
    assert t["kernel_hash"] == bench.kernel_hash()
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic() == t["das_hbm_bytes_per_launch"]


def test_kernel_hash_ignores_comments_only(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("// a kernel\n__global__ void k(float *x) { x[0] = 1.f; /* one */ }\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "KERNEL_SOURCES", ("k.hip",))
    h0 = bench.kernel_hash()
    src.write_text("// another comment\n__global__ void k(float *x) {\n  x[0] = 1.f;  // set\n}\n")
    assert bench.kernel_hash() == h0
    src.write_text("__global__ void k(float *x) { x[0] = 2.f; }\n")
    assert bench.kernel_hash() != h0


def test_stale_traffic_is_not_reported(tmp_path, monkeypatch):
    out = tmp_path / "traffic.json"
    out.write_text(json.dumps({"kernel_hash": "0" * 16, "das_hbm_bytes_per_launch": 123}))
    monkeypatch.setattr(bench, "TRAFFIC_FILE", str(out))
    assert bench.measured_traffic() is None


def test_roofline_objects():
    r = bench.alu_roofline(39.33, 1e9)
    assert r["bound"] == "alu" and r["peak"] == 157.3 and r["traffic"] == 1e9
    assert r["frac"] == pytest.approx(39.33 / 157.3, abs=1e-4)
    assert r["frac_nonpacked"] == pytest.approx(39.33 / bench.FP32_NONPACKED_TFLOPS, abs=1e-4)
    L = bench.lds_roofline(45_000_000_000, 68_700_000_000, 27.0)
    assert L["bound"] == "lds" and L["unit"] == "TB/s"
    assert L["achieved"] == pytest.approx(16 * 45e9 / 27e-3 / 1e12, abs=0.01)
    assert L["achieved_nominal"] == pytest.approx(16 * 68.7e9 / 27e-3 / 1e12, abs=0.01)
