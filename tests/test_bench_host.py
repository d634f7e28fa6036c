"""Host logic of the benchmark (CPU): the refusal of more than one GPU, the
roofline arithmetic of the fused step kernel, and the reading of the
committed counter summary, whose measured traffic is reported only for the
profiled configuration and only while the built library still has the hash
recorded with the counters."""
import hashlib
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=300)
    assert r.returncode == 2
    assert "one GPU" in r.stderr


def test_fused_roofline_arithmetic():
    r = dict(prec="f32", batch=128, kern_us=100.0, kern_n=10)
    roof = bench.fused_roofline(r, 240)
    flops = 128 * 4 * (240 * 241 // 2) * bench.FLOP_PER_ELEM_STAGE
    assert abs(roof["achieved"] - flops / 1e-4 / 1e12) < 1e-9
    assert abs(roof["frac"] - roof["achieved"] / 78.6) < 1e-12
    assert roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    assert abs(roof["hbm"]["algorithmic_bytes_per_launch"] - 128 * 240 * 240 * 22) < 1e-6
    assert bench.fused_roofline(dict(r, kern_us=0.0), 240) is None


def test_traffic_only_for_matching_library(tmp_path, monkeypatch):
    lib_dir = tmp_path / "paper_1609_03170_amd"
    lib_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    lib = lib_dir / "libopengrape.so"
    lib.write_bytes(b"\x7fELF built library")
    sha = hashlib.sha256(lib.read_bytes()).hexdigest()[:16]
    summary = tmp_path / bench.PROFILE
    summary.write_text("# summary\n\n| kernel | bytes |\n|---|---|\n\n"
                       f"traffic_bytes_per_launch: 123456\nlib-sha256-16: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("f32", 128, "banded") == 123456.0
    # other configurations have no counter summary
    assert bench.measured_traffic("f64", 128, "banded") is None
    assert bench.measured_traffic("f32", 64, "banded") is None
    assert bench.measured_traffic("f32", 128, "dense") is None
    assert bench.measured_traffic("f32", 128, "banded", fused=False) is None
    # a rebuilt library invalidates the counters
    lib.write_bytes(b"\x7fELF rebuilt library")
    assert bench.measured_traffic("f32", 128, "banded") is None
    # no summary at all
    lib.write_bytes(b"\x7fELF built library")
    summary.unlink()
    assert bench.measured_traffic("f32", 128, "banded") is None
