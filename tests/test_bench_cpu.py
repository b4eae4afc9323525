"""Host-side checks of bench.py that need no GPU: the one-GPU refusal, the
algorithmic byte model of each pass, and the traffic lookup's source-hash guard."""

import importlib.util
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def bench():
    spec = importlib.util.spec_from_file_location("bench_under_test", os.path.join(ROOT, "bench.py"))
    mod = importlib.util.module_from_spec(spec)
    spec.loader.exec_module(mod)
    return mod


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_kernel_bytes_model(bench):
    # the half spectrum is nz * ny * (nx/2 + 1) complex FP32 values, a real volume
    # nz * ny * nx FP32 values; each pass reads and writes what its design says
    nz, ny, nx = 4, 6, 8
    spec = nz * ny * (nx // 2 + 1) * 8
    real = nz * ny * nx * 4
    kb = bench.kernel_bytes((nz, ny, nx))
    assert kb["y"] == 2 * spec
    assert kb["z_otf"] == 3 * spec
    assert kb["x_ratio"] == 2 * spec + real
    assert kb["x_update"] == 2 * spec + 2 * real
    assert kb["x_update_last"] == spec + 2 * real
    assert kb["x_r2c"] == kb["x_c2r"] == spec + real


def test_traffic_lookup_requires_matching_source(bench, tmp_path, monkeypatch):
    good = (f"Kernel source sha256[:16]: `{bench.source_hash()}`.\n"
            "| per-launch HBM bytes (calibrated): 12345 | ratio to algorithmic 1.0 |\n")
    stale = good.replace(bench.source_hash(), "0" * 16)
    monkeypatch.setattr(bench, "PROFILES", str(tmp_path))
    (tmp_path / "traffic_y_w1.md").write_text(good)
    (tmp_path / "traffic_y_w2.md").write_text(stale)
    assert bench.measured_traffic("y", "w1") == 12345.0
    assert bench.measured_traffic("y", "w2") is None
    assert bench.measured_traffic("y", "w3") is None
