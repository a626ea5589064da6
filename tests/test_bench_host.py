"""Host logic of bench.py (no GPU): the one-GPU guard, the roofline record
of the dominant kernel and the staleness rule of the committed counter
tables."""
import hashlib
import json
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402


def test_more_than_one_gpu_exits_with_a_message():
    p = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert p.returncode == 2
    assert p.stdout.strip() == ""            # no JSON line
    assert "one GPU" in p.stderr


def _sizes():
    # sizes of the package-trace workload's model (only the keys stage_bytes reads)
    return {"Ng": 256 * 256 * 32, "n": 200_196, "b": 300_000, "l": 100_000, "nprime": 200_000,
            "nnz_near": 170_000_000}


def test_roofline_of_the_plane_kernel_is_its_alu_rate():
    R, grid = 512, (256, 256, 32)
    stages = {"fft_y": (110.0, 2), "project": (40.0, 2), "interp": (28.0, 2)}   # (ms, calls)
    roof = bench.roofline(stages, _sizes(), R, grid)
    assert roof["kernel"] == "k_fft_yz_big" and roof["bound"] == "alu" and roof["unit"] == "TFLOP/s"
    flops = 3 * R * 2 * grid[0] * bench.big_plane_flops(256, 32)
    assert roof["flops_per_launch"] == flops
    assert roof["achieved"] == pytest.approx(flops / 0.055 / 1e12, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.FP32_PEAK_TFLOPS, rel=1e-3)
    assert roof["frac_without_packed_fp32"] == pytest.approx(2 * roof["frac"], rel=1e-2)


def test_roofline_of_another_stage_is_its_hbm_rate():
    R, grid = 80, (256, 64, 32)
    stages = {"fft_y": (1.0, 1), "interp": (3.0, 1)}
    sz = _sizes()
    roof = bench.roofline(stages, sz, R, grid)
    assert roof["stage"] == "interp" and roof["bound"] == "hbm" and roof["unit"] == "GB/s"
    nb = bench.stage_bytes(sz, R)["interp"]
    assert roof["bytes_per_launch"] == nb
    assert roof["achieved"] == pytest.approx(nb / 3e-3 / 1e9, rel=1e-3)
    assert roof["frac"] == pytest.approx(roof["achieved"] / bench.HBM_PEAK_GBS, rel=1e-3)


def test_plane_flops_scale_with_the_transform_sizes():
    # per (channel, k_x) plane: doubling N_y adds one radix-2 level to each y
    # transform and doubles everything else
    a, b = bench.big_plane_flops(256, 32), bench.big_plane_flops(512, 32)
    assert 2 * a < b < 2.2 * a
    assert bench._fft(1) == 0 and bench._fft(8) == 5 * 8 * 3


def test_counter_table_is_dropped_when_its_sources_change(tmp_path, monkeypatch):
    src = tmp_path / "k.hip"
    src.write_text("kernel v1\n")
    (tmp_path / "profiles").mkdir()
    tab = {"sources_sha256": {"k.hip": hashlib.sha256(b"kernel v1\n").hexdigest()},
           "stages": {"fft_y": {"read_bytes": 10, "write_bytes": 5}},
           "step_read_bytes": 100, "step_write_bytes": 50}
    (tmp_path / "profiles" / "t.json").write_text(json.dumps(tab))
    monkeypatch.setattr(bench, "HERE", str(tmp_path))
    assert bench.measured_traffic("fft_y", "t") == 15
    assert bench.measured_traffic("interp", "t") is None
    assert bench.measured_step_bytes("t") == 150
    src.write_text("kernel v2\n")            # the kernel changed after the counters were taken
    assert bench.measured_traffic("fft_y", "t") is None
    assert bench.measured_step_bytes("t") is None
    assert bench.measured_traffic("fft_y", "absent") is None
