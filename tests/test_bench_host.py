"""Host logic of the benchmark (CPU): the refusal of more than one GPU, and
the reading of the committed counter summary, whose measured traffic is
reported only for the profiled configuration and only while the kernel
source still has the hash recorded with the counters."""
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


def test_traffic_only_for_matching_source(tmp_path, monkeypatch):
    src_dir = tmp_path / "paper_1609_03170_amd" / "csrc"
    src_dir.mkdir(parents=True)
    (tmp_path / "profiles").mkdir()
    src = src_dir / "og_device.h"
    src.write_text("// stage kernel source\n")
    sha = hashlib.sha256(src.read_bytes()).hexdigest()[:16]
    summary = tmp_path / "profiles" / "band_stage_kernel_transmon240_b128_f32.md"
    summary.write_text("# summary\n\n| kernel | bytes |\n|---|---|\n\n"
                       f"traffic_bytes_per_launch: 123456\nsource-sha256-16: {sha}\n")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    assert bench.measured_traffic("f32", 128, "banded") == 123456.0
    # other configurations have no counter summary
    assert bench.measured_traffic("f64", 128, "banded") is None
    assert bench.measured_traffic("f32", 64, "banded") is None
    assert bench.measured_traffic("f32", 128, "dense") is None
    # an edited kernel source invalidates the counters
    src.write_text("// stage kernel source, edited\n")
    assert bench.measured_traffic("f32", 128, "banded") is None
    # no summary at all
    src.write_text("// stage kernel source\n")
    summary.unlink()
    assert bench.measured_traffic("f32", 128, "banded") is None
