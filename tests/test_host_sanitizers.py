"""The C ABI's argument validation (rl_api.cpp) built with AddressSanitizer and
UndefinedBehaviorSanitizer on the host code and driven with invalid requests
(tests/sanitize/abi_driver.cpp).  The sanitizers instrument host code only; the
kernels' object is linked as built.  Runs on a host without a GPU (every request
is rejected before device work); skipped where the HIP toolchain or the built
kernels object is missing."""

import os
import shutil
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
PKG = os.path.join(ROOT, "paper_2510_14143_amd")
KOBJ = os.path.join(PKG, "_build", "rl_kernels.o")
HIPCC = "/opt/rocm/bin/hipcc"
SAN = ["-Xarch_host", "-fsanitize=address", "-Xarch_host", "-fsanitize=undefined",
       "-Xarch_host", "-fno-sanitize-recover=undefined", "-fno-omit-frame-pointer"]


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


@pytest.mark.slow
@pytest.mark.skipif(not os.path.exists(HIPCC) or not os.path.exists(KOBJ),
                    reason="needs hipcc and the built kernels object")
@pytest.mark.skipif(_has_gpu(), reason="drives the no-device validation path")
def test_validation_layer_under_asan_and_ubsan(tmp_path):
    common = ["--offload-arch=gfx950", "-O1", "-g", "-std=c++17", "-fPIC",
              "-Wno-unused-command-line-argument", "-I", os.path.join(ROOT, "include"),
              "-I", os.path.join(PKG, "csrc")]
    api = tmp_path / "rl_api.o"
    drv = tmp_path / "driver.o"
    exe = tmp_path / "abi_driver"
    subprocess.run([HIPCC, *common, *SAN, "-x", "hip", "-c", os.path.join(PKG, "csrc", "rl_api.cpp"),
                    "-o", str(api)], check=True, timeout=900)
    subprocess.run([HIPCC, *common, *SAN, "-c", os.path.join(ROOT, "tests", "sanitize",
                                                             "abi_driver.cpp"), "-o", str(drv)],
                   check=True, timeout=900)
    subprocess.run([HIPCC, "--offload-arch=gfx950", *SAN, str(api), KOBJ, str(drv), "-o", str(exe),
                    "-L/opt/rocm/lib", "-lrocprofiler-sdk-roctx"], check=True, timeout=900)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([str(exe)], capture_output=True, text=True, timeout=300, env=env)
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.strip().endswith("OK"), r.stdout
    assert "runtime error" not in r.stderr and "AddressSanitizer" not in r.stderr, r.stderr
