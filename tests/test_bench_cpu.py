"""Host-side checks of bench.py that need no GPU: the one-GPU refusal, the
algorithmic byte model of each pass, the guard around the secondary workloads, and
the rocprofv3 summary step (CSV parsing, back-to-back launches, counter
calibration, the source-hash guard)."""

import importlib.util
import os
import subprocess
import sys

import numpy as np
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


def test_optional_leg_records_a_failure(bench, capsys):
    # a secondary workload that fails is logged and recorded in its place; the
    # others (and the headline line) go on
    assert bench.optional_leg("fine", lambda: {"value": 1.0}) == {"value": 1.0}

    def broken():
        raise RuntimeError("no memory left")

    rec = bench.optional_leg("broken", broken)
    assert rec == {"error": "RuntimeError: no memory left"}
    err = capsys.readouterr().err
    assert "broken failed" in err and "Traceback" in err


def test_kernel_short_name(bench):
    assert bench.kernel_short_name(
        "void rlmi::k_pencil<8, 0, 1024, 0>(HIP_vector_type<float, 2u>*, rlmi::PencilArgs)"
    ) == "k_pencil<8, 0, 1024, 0>"
    assert bench.kernel_short_name("rlmi::k_xrow<4, 2, 0>(rlmi::XArgs)") == "k_xrow<4, 2, 0>"
    assert bench.kernel_short_name("k_copy(float4 const*, float4*, long long)") == "k_copy"
    assert bench.kernel_short_name(
        "void at::native::kern<4, at::F<float>, std::array<char*, 1ul> >(int)"
    ) == "kern<4, at::F<float>, std::array<char*, 1ul> >"


def _write_csv(path, header, rows):
    path.parent.mkdir(parents=True, exist_ok=True)
    with open(path, "w") as f:
        f.write(",".join(f'"{h}"' for h in header) + "\n")
        for r in rows:
            f.write(",".join(f'"{v}"' for v in r) + "\n")


def _fixture(tmp_path):
    """A kernel trace and two counter runs of a made-up profiled command: two copy
    launches, five Y launches (three back to back), one other kernel in between."""
    y = "void rlmi::k_pencil<8, 0, 1024, 0>(HIP_vector_type<float, 2u>*, rlmi::PencilArgs)"
    cp = "void rlmi::k_copy(HIP_vector_type<float, 4u> const*, HIP_vector_type<float, 4u>*, long long)"
    other = "void rlmi::k_xrow<4, 2, 0>(rlmi::XArgs, rlmi::Sched, HIP_vector_type<float, 2u> const*)"
    hdr = ["Kind", "Agent_Id", "Queue_Id", "Kernel_Id", "Kernel_Name", "Correlation_Id",
           "Start_Timestamp", "End_Timestamp", "Workgroup_Size_X", "Workgroup_Size_Y",
           "Workgroup_Size_Z", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z"]
    launches = [  # (name, start, end, grid x); times in ns
        (cp, 0, 400_000, 4096), (cp, 500_000, 900_000, 4096),
        (y, 1_000_000, 1_100_000, 8192),   # after a 100 us gap: not back to back
        (y, 1_100_500, 1_200_500, 8192),   # 0.5 us gap: back to back, 100 us
        (other, 1_200_800, 1_230_800, 1024),
        (y, 1_231_000, 1_341_000, 8192),   # back to back, 110 us
        (y, 1_341_200, 1_461_200, 8192),   # back to back, 120 us
        (y, 1_600_000, 1_690_000, 8192),   # 139 us gap: not back to back, 90 us
    ]
    rows = [["KERNEL_DISPATCH", 1, 7, i, n, i, s, e, 256, 1, 1, g, 1, 1]
            for i, (n, s, e, g) in enumerate(launches)]
    _write_csv(tmp_path / "trace" / "host" / "1" / "run_kernel_trace.csv", hdr, rows)
    chdr = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
            "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "Counter_Name",
            "Counter_Value"]
    # the copy moves 1 GiB each way: FETCH_SIZE reads half of it (x2), WRITE_SIZE all of it
    fetch = [[1, 1, 1, 7, 1, 1, 4096, 1, cp, 256, "FETCH_SIZE", (1 << 30) / 1024 / 2],
             [2, 2, 1, 7, 1, 1, 8192, 2, y, 256, "FETCH_SIZE", 1000.0],
             [3, 3, 1, 7, 1, 1, 8192, 2, y, 256, "FETCH_SIZE", 3000.0]]
    write = [[1, 1, 1, 7, 1, 1, 4096, 1, cp, 256, "WRITE_SIZE", (1 << 30) / 1024],
             [2, 2, 1, 7, 1, 1, 8192, 2, y, 256, "WRITE_SIZE", 500.0]]
    _write_csv(tmp_path / "fetch" / "run_counter_collection.csv", chdr, fetch)
    _write_csv(tmp_path / "write" / "run_counter_collection.csv", chdr, write)
    return "k_pencil<8, 0, 1024, 0>"


def test_rocprof_summary_and_lookup(bench, tmp_path, monkeypatch):
    yname = _fixture(tmp_path)
    text = bench.rocprof_summary(str(tmp_path / "trace"), str(tmp_path / "fetch"),
                                 str(tmp_path / "write"), "fixture", ["cmd one", "cmd two"])
    assert "FETCH_SIZE x2.000, WRITE_SIZE x1.000" in text
    assert "    cmd one" in text
    prof = tmp_path / "profiles"
    prof.mkdir()
    monkeypatch.setattr(bench, "PROFILES", str(prof))
    (prof / "kernel_trace_w1.md").write_text(text)
    rows = bench.read_summary(bench.summary_path("w1"))
    y = rows[(yname, 8192)]
    assert y["n"] == 5 and y["nb"] == 3
    assert y["avg_us"] == pytest.approx((100 + 100 + 110 + 120 + 90) / 5)
    assert y["b2b_us"] == pytest.approx((100 + 110 + 120) / 3)
    assert y["read"] == pytest.approx(2000.0 * 1024 * 2)   # mean 2000 KiB, x2 calibration
    assert y["write"] == pytest.approx(500.0 * 1024)
    assert rows[("k_copy", 4096)]["read"] == pytest.approx(1 << 30)
    other = rows[("k_xrow<4, 2, 0>", 1024)]
    assert other["nb"] == 1 and np.isnan(other["read"])
    fig = bench.trace_figures(bench.summary_path("w1"), [yname, "k_pencil<8, 1, 1024, 0>"], 8192)
    assert fig["b2b_us"] == pytest.approx(110.0) and fig["b2b_launches"] == 3
    assert fig["traffic"] == pytest.approx(2000.0 * 1024 * 2 + 500.0 * 1024)
    assert bench.trace_figures(bench.summary_path("w1"), [yname], 4096) is None
    # a summary taken on another kernel source is not used
    (prof / "kernel_trace_w2.md").write_text(text.replace(bench.source_hash(), "0" * 16))
    assert bench.read_summary(bench.summary_path("w2")) is None
    assert bench.trace_figures(bench.summary_path("w2"), [yname], 8192) is None
    assert bench.trace_figures(bench.summary_path("w3"), [yname], 8192) is None


def test_rocprof_summary_command_line(tmp_path):
    _fixture(tmp_path)
    out = tmp_path / "s.md"
    log = tmp_path / "bench.err"
    log.write_text("copy probe: 5500 GB/s\nkernel source sha256[:16]: 0123456789abcdef\n")
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--rocprof-summary",
                        str(tmp_path / "trace"), str(tmp_path / "fetch"), str(tmp_path / "write"),
                        "--out", str(out), "--title", "t", "--cmd", "c", "--bench-log", str(log)],
                       capture_output=True, text=True, timeout=300, cwd=ROOT)
    assert r.returncode == 0, r.stderr
    text = out.read_text()
    assert "| `k_copy` | 4096 | 2 |" in text
    # the hash is the one the profiled run reported, not the current source's
    assert "Kernel source sha256[:16]: `0123456789abcdef`" in text
