"""C-ABI checks that need no GPU: the library loads, exports every declared
symbol, and rejects bad arguments with the documented status codes before any
device work."""

import ctypes

import pytest

from paper_2510_14143_amd import rl


def _has_gpu():
    try:
        import torch
        return torch.cuda.is_available()
    except Exception:
        return False


def test_library_exports_every_declared_symbol():
    names = rl.header_functions()
    assert {"rl_plan_create", "rl_iterate", "conv3d_fft", "rl_plan_destroy"} <= set(names)
    L = rl.lib()
    for n in names:
        assert hasattr(L, n), n


def _create(shape, psf_ptr=4096, boundary=0):
    out = ctypes.c_void_p(1234)
    sh = (ctypes.c_int64 * 3)(*shape)
    st = rl.lib().rl_plan_create(sh, ctypes.c_void_p(psf_ptr), boundary, ctypes.byref(out))
    return st, out.value


@pytest.mark.parametrize("shape,code", [
    ((0, 8, 8), rl.RL_E_INVALID),
    ((8, -1, 8), rl.RL_E_INVALID),
    ((8, 8, 7), rl.RL_E_UNSUPPORTED),      # odd nx
    ((8, 8, 2), rl.RL_E_UNSUPPORTED),      # nx < 4
    ((8, 8, 22), rl.RL_E_UNSUPPORTED),     # radix 11
    ((8, 26, 8), rl.RL_E_UNSUPPORTED),     # radix 13
    ((8, 8, 54), rl.RL_E_UNSUPPORTED),     # nx/2 = 27: the X rule needs the odd part in one thread
    ((8, 22, 8), rl.RL_E_UNSUPPORTED),     # radix 11 in Y
    ((8, 8, 70), rl.RL_E_UNSUPPORTED),     # nx/2 = 35 = 5 * 7
    ((8, 105, 8), rl.RL_E_UNSUPPORTED),    # 3 * 5 * 7: no element count holds all three primes
    ((8, 8, 8192), rl.RL_E_UNSUPPORTED),   # above the nx limit
    ((8, 8, 4096), rl.RL_E_UNSUPPORTED),   # nx/2 = 2048 needs 32 elements per thread
    ((8192, 8, 8), rl.RL_E_UNSUPPORTED),   # above the nz limit
    ((8, 8192, 8), rl.RL_E_UNSUPPORTED),   # above the ny limit
])
def test_bad_shapes_rejected(shape, code):
    st, out = _create(shape)
    assert st == code, rl.rl_last_error()
    assert out is None  # *out is cleared on failure


def test_bad_arguments_rejected():
    L = rl.lib()
    sh = (ctypes.c_int64 * 3)(8, 8, 8)
    out = ctypes.c_void_p()
    assert L.rl_plan_create(None, ctypes.c_void_p(4096), 0, ctypes.byref(out)) == rl.RL_E_INVALID
    assert L.rl_plan_create(sh, ctypes.c_void_p(4096), 0, None) == rl.RL_E_INVALID
    assert L.rl_plan_create(sh, None, 0, ctypes.byref(out)) == rl.RL_E_INVALID
    assert L.rl_plan_create(sh, ctypes.c_void_p(4100), 0, ctypes.byref(out)) == rl.RL_E_INVALID
    assert L.rl_plan_create(sh, ctypes.c_void_p(4096), 7, ctypes.byref(out)) == rl.RL_E_INVALID
    # zero boundary: the padded grid must be supported (nx 3000 pads beyond 4096)
    big = (ctypes.c_int64 * 3)(8, 8, 3000)
    assert L.rl_plan_create(big, ctypes.c_void_p(4096), rl.RL_BOUNDARY_ZERO,
                            ctypes.byref(out)) == rl.RL_E_UNSUPPORTED
    assert "zero boundary" in rl.rl_last_error()
    # psf_shape must lie in [1, volume dimension]
    for ps in ((9, 8, 8), (8, -1, 8), (8, 8, 9)):
        opt = rl._Options(0, None, 0, 0, 0, 0, 0, (ctypes.c_int64 * 3)(*ps))
        st = L.rl_plan_create_ex(sh, ctypes.c_void_p(4096), 0, ctypes.byref(opt), ctypes.byref(out))
        assert st == rl.RL_E_INVALID and "psf_shape" in rl.rl_last_error(), ps
    # batch plans: periodic boundary, same-shape PSFs
    ps = (ctypes.c_void_p * 1)(4096)
    assert L.rl_plan_create_batch(1, sh, ps, rl.RL_BOUNDARY_ZERO, None,
                                  ctypes.byref(out)) == rl.RL_E_UNSUPPORTED


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
@pytest.mark.parametrize("shape", [(7, 9, 11), (1, 5, 3), (30, 100, 90)])
def test_zero_boundary_accepts_any_volume_shape(shape):
    # every dimension is allowed with the zero boundary (the grid is padded); without a
    # device the call gets as far as the device check
    st, out = _create(shape, boundary=rl.RL_BOUNDARY_ZERO)
    assert st == rl.RL_E_DEVICE, rl.rl_last_error()


@pytest.mark.skipif(_has_gpu(), reason="checks the no-device path")
def test_no_device_is_reported():
    st, out = _create((8, 8, 8))
    assert st == rl.RL_E_DEVICE
    assert out is None


def test_handles_are_checked_without_dereference():
    L = rl.lib()
    fake = ctypes.c_void_p(0x1234560)
    assert L.rl_iterate(None, None, None, 1) == rl.RL_E_INVALID
    assert L.rl_iterate(fake, None, None, 1) == rl.RL_E_INVALID
    assert "live plan" in rl.rl_last_error()
    assert L.conv3d_fft(fake, None, None) == rl.RL_E_INVALID
    assert L.rl_plan_set_stream(fake, None) == rl.RL_E_INVALID
    n = ctypes.c_int()
    assert L.rl_plan_get_flux(fake, None, 0, ctypes.byref(n)) == rl.RL_E_INVALID
    ms = ctypes.c_double()
    assert L.rl_plan_time_pass(fake, 4, None, None, 1, ctypes.byref(ms)) == rl.RL_E_INVALID
    L.rl_plan_destroy(None)
    L.rl_plan_destroy(fake)  # unknown handle: ignored


def test_probe_copy_validation():
    L = rl.lib()
    assert L.rl_probe_copy(None, None, 0, None) == rl.RL_OK
    assert L.rl_probe_copy(ctypes.c_void_p(4096), ctypes.c_void_p(8192), 10, None) == rl.RL_E_INVALID
    assert L.rl_probe_copy(None, ctypes.c_void_p(8192), 16, None) == rl.RL_E_INVALID


def test_status_strings():
    assert rl.rl_status_string(rl.RL_OK) == "RL_OK"
    assert rl.rl_status_string(rl.RL_E_NUMERIC) == "RL_E_NUMERIC"
    assert rl.rl_status_string(99) == "RL_E_UNKNOWN"


def test_python_errors_carry_status():
    with pytest.raises(rl.RLError) as ei:
        rl.rl_plan_create((8, 8, 7), 4096)
    assert ei.value.status == rl.RL_E_UNSUPPORTED
    with pytest.raises(rl.RLError) as ei:
        rl.rl_iterate(0x1234560, 0, 0, 1)
    assert ei.value.status == rl.RL_E_INVALID


def test_elems_options_validated_before_device_work():
    L = rl.lib()
    sh = (ctypes.c_int64 * 3)(8, 16, 32)
    out = ctypes.c_void_p()
    for xe, yze in ((5, 0), (3, 0), (32, 0), (0, 3), (0, 7), (1, 0)):
        opt = rl._Options(0, None, 0, xe, yze)
        st = L.rl_plan_create_ex(sh, ctypes.c_void_p(4096), 0, ctypes.byref(opt), ctypes.byref(out))
        assert st == rl.RL_E_INVALID, (xe, yze, rl.rl_last_error())
    for accel in (-1, 2, 7):
        opt = rl._Options(0, None, 0, 0, 0, 0, accel)
        st = L.rl_plan_create_ex(sh, ctypes.c_void_p(4096), 0, ctypes.byref(opt), ctypes.byref(out))
        assert st == rl.RL_E_INVALID and "accel" in rl.rl_last_error()


def test_fsc_and_split_validation():
    L = rl.lib()
    curve = (ctypes.c_double * 9)()
    fake = ctypes.c_void_p(0x1234560)
    assert L.rl_fsc(fake, None, None, 8, 0.1, curve, None) == rl.RL_E_INVALID
    for shape in ((3, 4, 4), (4, 0, 4), (4, 4, 5)):
        sh = (ctypes.c_int64 * 3)(*shape)
        assert L.rl_split_diagonal(ctypes.c_void_p(4096), sh, ctypes.c_void_p(4096),
                                   ctypes.c_void_p(4096), None) == rl.RL_E_INVALID
    assert L.rl_split_diagonal(None, None, None, None, None) == rl.RL_E_INVALID


def test_ssim_checks_handle():
    L = rl.lib()
    v = ctypes.c_double()
    assert L.rl_ssim(ctypes.c_void_p(0x1234560), None, None, ctypes.byref(v)) == rl.RL_E_INVALID


def test_alpha_query_checks_handle():
    L = rl.lib()
    n = ctypes.c_int()
    assert L.rl_plan_get_alpha(ctypes.c_void_p(0x1234560), None, 0, ctypes.byref(n)) == rl.RL_E_INVALID


def test_missing_library_fails_loudly(monkeypatch, tmp_path):
    # with the HIP library absent, the binding raises; there is no fallback path
    monkeypatch.setattr(rl, "_lib", None)
    monkeypatch.setattr(rl, "LIB_PATH", str(tmp_path / "librlmi.so"))
    with pytest.raises(RuntimeError, match="is not built"):
        rl.lib()
    with pytest.raises(RuntimeError, match="is not built"):
        rl.rl_plan_create((8, 8, 8), 4096)
