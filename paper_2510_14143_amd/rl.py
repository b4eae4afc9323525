"""Python binding of librlmi.so: the C ABI of include/rl.h, one function per entry point.

The functions here only marshal arguments (ints and device pointers) and turn
status codes into RLError; every step of the computation runs in the HIP
kernels of the library.  `Plan` wraps them for torch tensors: it checks dtype,
device, shape and contiguity, and enqueues on torch's current stream.

The library is loaded on first use; if it has not been built, the first call
raises (there is no fallback implementation).
"""

from __future__ import annotations

import ctypes
import os
import re

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "librlmi.so")
HEADER_PATH = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))),
                           "include", "rl.h")

RL_OK, RL_E_INVALID, RL_E_UNSUPPORTED, RL_E_NOMEM, RL_E_DEVICE, RL_E_NUMERIC, RL_E_INTERNAL = range(7)
RL_BOUNDARY_PERIODIC, RL_BOUNDARY_ZERO = 0, 1
RL_PRECISION_FP32, RL_PRECISION_SPLIT_BF16, RL_PRECISION_SPLIT_FP16 = 0, 1, 2
_PRECISIONS = {"fp32": RL_PRECISION_FP32, "split_bf16": RL_PRECISION_SPLIT_BF16,
               "split_fp16": RL_PRECISION_SPLIT_FP16}
RL_ACCEL_NONE, RL_ACCEL_BIGGS_ANDREWS = 0, 1
RL_STOP_LOGLIK, RL_STOP_CHANGE, RL_STOP_PSNR, RL_STOP_SSIM, RL_STOP_FSC = 1, 2, 3, 4, 5
_STOP_METRICS = {"loglik": RL_STOP_LOGLIK, "change": RL_STOP_CHANGE, "psnr": RL_STOP_PSNR,
                 "ssim": RL_STOP_SSIM, "fsc": RL_STOP_FSC}
_ACCELS = {"none": RL_ACCEL_NONE, "biggs_andrews": RL_ACCEL_BIGGS_ANDREWS}
KERNEL_KINDS = ("x_r2c", "x_c2r", "x_ratio", "x_update", "y", "z_otf", "z", "other")


class RLError(RuntimeError):
    """A non-OK status from the library; .status holds the code."""

    def __init__(self, status: int, message: str):
        super().__init__(f"{_STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


_STATUS_NAMES = {0: "RL_OK", 1: "RL_E_INVALID", 2: "RL_E_UNSUPPORTED", 3: "RL_E_NOMEM",
                 4: "RL_E_DEVICE", 5: "RL_E_NUMERIC", 6: "RL_E_INTERNAL"}


class _StopRule(ctypes.Structure):
    _fields_ = [("metric", ctypes.c_int), ("threshold", ctypes.c_double), ("min_iter", ctypes.c_int),
                ("reference", ctypes.c_void_p), ("fsc_bins", ctypes.c_int),
                ("fsc_threshold", ctypes.c_double)]


class _Options(ctypes.Structure):
    _fields_ = [("precision", ctypes.c_int), ("stream", ctypes.c_void_p), ("tile_x", ctypes.c_int),
                ("x_elems", ctypes.c_int), ("yz_elems", ctypes.c_int), ("autotune", ctypes.c_int),
                ("accel", ctypes.c_int), ("psf_shape", ctypes.c_int64 * 3),
                ("batch_mode", ctypes.c_int)]


_lib = None


def lib() -> ctypes.CDLL:
    """Load librlmi.so (once).  Raises if it is not built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is not built; run `python -m paper_2510_14143_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp, i64p = ctypes.c_void_p, ctypes.POINTER(ctypes.c_int64)
    sig = {
        "rl_plan_create": ([i64p, vp, ctypes.c_int, ctypes.POINTER(vp)], ctypes.c_int),
        "rl_plan_create_ex": ([i64p, vp, ctypes.c_int, ctypes.POINTER(_Options), ctypes.POINTER(vp)],
                              ctypes.c_int),
        "rl_iterate": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "rl_iterate_noalloc": ([vp, vp, vp, ctypes.c_int], ctypes.c_int),
        "conv3d_fft": ([vp, vp, vp], ctypes.c_int),
        "rl_plan_destroy": ([vp], None),
        "rl_plan_set_stream": ([vp, vp], ctypes.c_int),
        "rl_plan_get_flux": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                              ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rl_plan_get_alpha": ([vp, ctypes.POINTER(ctypes.c_double), ctypes.c_int,
                               ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rl_plan_get_info": ([vp, i64p, i64p], ctypes.c_int),
        "rl_plan_get_grid": ([vp, i64p], ctypes.c_int),
        "rl_iterate_stop": ([vp, vp, vp, ctypes.c_int, ctypes.POINTER(_StopRule)], ctypes.c_int),
        "rl_ssim": ([vp, vp, vp, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "rl_fsc": ([vp, vp, vp, ctypes.c_int, ctypes.c_double, ctypes.POINTER(ctypes.c_double),
                    ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "rl_split_diagonal": ([vp, i64p, vp, vp, vp], ctypes.c_int),
        "rl_plan_get_stop": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double),
                              ctypes.c_int, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rl_plan_get_launch": ([vp, ctypes.POINTER(ctypes.c_int)], ctypes.c_int),
        "rl_plan_set_timing": ([vp, ctypes.c_int], ctypes.c_int),
        "rl_plan_time_pass": ([vp, ctypes.c_int, vp, vp, ctypes.c_int,
                               ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
        "rl_plan_get_timing": ([vp, ctypes.POINTER(ctypes.c_int), ctypes.POINTER(ctypes.c_double)],
                               ctypes.c_int),
        "rl_plan_get_pass_kernel": ([vp, ctypes.c_int, ctypes.c_char_p, ctypes.c_size_t, i64p],
                                    ctypes.c_int),
        "rl_probe_copy": ([vp, vp, ctypes.c_size_t, vp], ctypes.c_int),
        "rl_plan_create_batch": ([ctypes.c_int, i64p, ctypes.POINTER(vp), ctypes.c_int,
                                  ctypes.POINTER(_Options), ctypes.POINTER(vp)], ctypes.c_int),
        "rl_iterate_batch": ([vp, ctypes.POINTER(vp), ctypes.POINTER(vp), ctypes.c_int],
                             ctypes.c_int),
        "rl_status_string": ([ctypes.c_int], ctypes.c_char_p),
        "rl_last_error": ([], ctypes.c_char_p),
    }
    for name, (args, res) in sig.items():
        fn = getattr(L, name)
        fn.argtypes = args
        fn.restype = res
    _lib = L
    return L


def header_functions() -> list:
    """Names of the functions declared in include/rl.h."""
    with open(HEADER_PATH) as f:
        text = re.sub(r"/\*.*?\*/", "", f.read(), flags=re.S)
    return re.findall(r"^[A-Za-z_][\w\s\*]*?\b(rl_\w+|conv3d_fft)\s*\(", text, flags=re.M)


def _check(st: int) -> None:
    if st != RL_OK:
        msg = lib().rl_last_error().decode(errors="replace")
        raise RLError(st, msg)


def _shape(shape) -> ctypes.Array:
    if len(shape) != 3:
        raise ValueError("shape must be (nz, ny, nx)")
    return (ctypes.c_int64 * 3)(*[int(s) for s in shape])


# ---------------------------------------------------------------------------
# one function per C entry point
# ---------------------------------------------------------------------------

def rl_plan_create(shape, psf_ptr: int, boundary: int = RL_BOUNDARY_PERIODIC) -> int:
    out = ctypes.c_void_p()
    _check(lib().rl_plan_create(_shape(shape), ctypes.c_void_p(psf_ptr), int(boundary),
                                ctypes.byref(out)))
    return out.value


def rl_plan_create_ex(shape, psf_ptr: int, boundary: int = RL_BOUNDARY_PERIODIC,
                      precision: int = RL_PRECISION_FP32, stream: int = 0, tile_x: int = 0,
                      x_elems: int = 0, yz_elems: int = 0, autotune: bool = False,
                      accel: int = RL_ACCEL_NONE, psf_shape=(0, 0, 0)) -> int:
    out = ctypes.c_void_p()
    opt = _Options(int(precision), ctypes.c_void_p(stream or None), int(tile_x), int(x_elems),
                   int(yz_elems), 1 if autotune else 0, int(accel),
                   (ctypes.c_int64 * 3)(*[int(v) for v in psf_shape]))
    _check(lib().rl_plan_create_ex(_shape(shape), ctypes.c_void_p(psf_ptr), int(boundary),
                                   ctypes.byref(opt), ctypes.byref(out)))
    return out.value


def rl_iterate(plan: int, observed_ptr: int, estimate_ptr: int, n_iter: int) -> None:
    _check(lib().rl_iterate(ctypes.c_void_p(plan), ctypes.c_void_p(observed_ptr),
                            ctypes.c_void_p(estimate_ptr), int(n_iter)))


def rl_iterate_noalloc(plan: int, observed_ptr: int, estimate_ptr: int, n_iter: int) -> None:
    _check(lib().rl_iterate_noalloc(ctypes.c_void_p(plan), ctypes.c_void_p(observed_ptr),
                                    ctypes.c_void_p(estimate_ptr), int(n_iter)))


def conv3d_fft(plan: int, x_ptr: int, out_ptr: int) -> None:
    _check(lib().conv3d_fft(ctypes.c_void_p(plan), ctypes.c_void_p(x_ptr), ctypes.c_void_p(out_ptr)))


RL_BATCH_AUTO, RL_BATCH_PERSISTENT, RL_BATCH_GRAPH = 0, 1, 2
_BATCH_MODES = {"auto": RL_BATCH_AUTO, "persistent": RL_BATCH_PERSISTENT, "graph": RL_BATCH_GRAPH}


def rl_plan_create_batch(shapes, psf_ptrs, boundary: int = RL_BOUNDARY_PERIODIC,
                         stream: int = 0, x_elems: int = 0, yz_elems: int = 0,
                         autotune: bool = False, batch_mode: int = RL_BATCH_AUTO) -> int:
    n = len(shapes)
    if len(psf_ptrs) != n:
        raise ValueError("one PSF per volume")
    sh = (ctypes.c_int64 * (3 * n))(*[int(v) for s3 in shapes for v in s3])
    ps = (ctypes.c_void_p * n)(*psf_ptrs)
    out = ctypes.c_void_p()
    opt = _Options(RL_PRECISION_FP32, ctypes.c_void_p(stream or None), 0, int(x_elems),
                   int(yz_elems), 1 if autotune else 0, RL_ACCEL_NONE,
                   (ctypes.c_int64 * 3)(0, 0, 0), int(batch_mode))
    _check(lib().rl_plan_create_batch(n, sh, ps, int(boundary), ctypes.byref(opt),
                                      ctypes.byref(out)))
    return out.value


def rl_iterate_batch(plan: int, observed_ptrs, estimate_ptrs, n_iter: int) -> None:
    n = len(observed_ptrs)
    ob = (ctypes.c_void_p * n)(*observed_ptrs)
    es = (ctypes.c_void_p * n)(*estimate_ptrs)
    _check(lib().rl_iterate_batch(ctypes.c_void_p(plan), ob, es, int(n_iter)))


def rl_plan_destroy(plan: int) -> None:
    lib().rl_plan_destroy(ctypes.c_void_p(plan))


def rl_plan_set_stream(plan: int, stream: int) -> None:
    _check(lib().rl_plan_set_stream(ctypes.c_void_p(plan), ctypes.c_void_p(stream or None)))


def rl_plan_get_flux(plan: int, cap: int = 1 << 20) -> np.ndarray:
    n = ctypes.c_int(0)
    _check(lib().rl_plan_get_flux(ctypes.c_void_p(plan), None, 0, ctypes.byref(n)))
    buf = (ctypes.c_double * max(1, n.value))()
    m = ctypes.c_int(0)
    st = lib().rl_plan_get_flux(ctypes.c_void_p(plan), buf, min(cap, n.value), ctypes.byref(m))
    vals = np.array(buf[: min(cap, m.value)], dtype=np.float64)
    _check(st)
    return vals


def rl_plan_get_alpha(plan: int) -> np.ndarray:
    n = ctypes.c_int(0)
    _check(lib().rl_plan_get_alpha(ctypes.c_void_p(plan), None, 0, ctypes.byref(n)))
    buf = (ctypes.c_double * max(1, n.value))()
    _check(lib().rl_plan_get_alpha(ctypes.c_void_p(plan), buf, n.value, ctypes.byref(n)))
    return np.array(buf[: n.value], dtype=np.float64)


def rl_iterate_stop(plan: int, observed_ptr: int, estimate_ptr: int, max_iter: int, metric: int,
                    threshold: float, min_iter: int = 0, reference_ptr: int = 0,
                    fsc_bins: int = 0, fsc_threshold: float = 0.0) -> None:
    rule = _StopRule(int(metric), float(threshold), int(min_iter),
                     ctypes.c_void_p(reference_ptr or None), int(fsc_bins), float(fsc_threshold))
    _check(lib().rl_iterate_stop(ctypes.c_void_p(plan), ctypes.c_void_p(observed_ptr),
                                 ctypes.c_void_p(estimate_ptr), int(max_iter), ctypes.byref(rule)))


def rl_plan_get_stop(plan: int):
    """(iterations done, metric history) of the last rl_iterate_stop call."""
    n_done, n_hist = ctypes.c_int(0), ctypes.c_int(0)
    _check(lib().rl_plan_get_stop(ctypes.c_void_p(plan), ctypes.byref(n_done), None, 0,
                                  ctypes.byref(n_hist)))
    buf = (ctypes.c_double * max(1, n_hist.value))()
    _check(lib().rl_plan_get_stop(ctypes.c_void_p(plan), ctypes.byref(n_done), buf, n_hist.value,
                                  ctypes.byref(n_hist)))
    return n_done.value, np.array(buf[: n_hist.value], dtype=np.float64)


def rl_ssim(plan: int, u_ptr: int, ref_ptr: int) -> float:
    v = ctypes.c_double(0.0)
    _check(lib().rl_ssim(ctypes.c_void_p(plan), ctypes.c_void_p(u_ptr), ctypes.c_void_p(ref_ptr),
                         ctypes.byref(v)))
    return v.value


def rl_fsc(plan: int, a_ptr: int, b_ptr: int, nbins: int = 64, threshold: float = 1.0 / 7.0):
    """(FSC curve over nbins + 1 shells, resolution in cycles per voxel)."""
    curve = (ctypes.c_double * (nbins + 1))()
    res = ctypes.c_double(0.0)
    _check(lib().rl_fsc(ctypes.c_void_p(plan), ctypes.c_void_p(a_ptr), ctypes.c_void_p(b_ptr),
                        int(nbins), float(threshold), curve, ctypes.byref(res)))
    return np.array(curve[:], dtype=np.float64), res.value


def rl_split_diagonal(u_ptr: int, shape, a_ptr: int, b_ptr: int, stream: int = 0) -> None:
    _check(lib().rl_split_diagonal(ctypes.c_void_p(u_ptr), _shape(shape), ctypes.c_void_p(a_ptr),
                                   ctypes.c_void_p(b_ptr), ctypes.c_void_p(stream or None)))


def split_diagonal(u):
    """The two diagonal half-size sub-volumes of u (new tensors)."""
    import torch
    if u.dim() != 3:
        raise ValueError("u must be a 3-D tensor")
    _check_volume(u, u.shape, None, "u")
    half = tuple(int(n) // 2 for n in u.shape)
    a = torch.empty(half, dtype=torch.float32, device=u.device)
    b = torch.empty_like(a)
    rl_split_diagonal(u.data_ptr(), tuple(u.shape), a.data_ptr(), b.data_ptr(), _stream_of(u.device))
    return a, b


def rl_plan_get_grid(plan: int) -> tuple:
    g = (ctypes.c_int64 * 3)()
    _check(lib().rl_plan_get_grid(ctypes.c_void_p(plan), g))
    return tuple(int(v) for v in g)


def rl_plan_get_info(plan: int):
    shape = (ctypes.c_int64 * 3)()
    pitch = ctypes.c_int64(0)
    _check(lib().rl_plan_get_info(ctypes.c_void_p(plan), shape, ctypes.byref(pitch)))
    return tuple(shape), pitch.value


def rl_plan_get_launch(plan: int) -> dict:
    out = (ctypes.c_int * 8)()
    _check(lib().rl_plan_get_launch(ctypes.c_void_p(plan), out))
    return dict(x_elems=out[0], y_elems=out[1], y_lanes=out[2], z_elems=out[3], z_lanes=out[4],
                tuned=bool(out[5]), z_rows_fastest=bool(out[6]), batch_persistent=bool(out[7]))


def rl_plan_set_timing(plan: int, enable: bool) -> None:
    _check(lib().rl_plan_set_timing(ctypes.c_void_p(plan), 1 if enable else 0))


def rl_plan_get_timing(plan: int) -> dict:
    cnt = (ctypes.c_int * len(KERNEL_KINDS))()
    ms = (ctypes.c_double * len(KERNEL_KINDS))()
    _check(lib().rl_plan_get_timing(ctypes.c_void_p(plan), cnt, ms))
    return {k: (cnt[i], ms[i]) for i, k in enumerate(KERNEL_KINDS)}


def rl_plan_time_pass(plan: int, kind: str, observed_ptr: int, estimate_ptr: int,
                      reps: int = 20) -> float:
    """Average ms per launch of one pass kind over a burst of `reps` launches."""
    ms = ctypes.c_double(0.0)
    _check(lib().rl_plan_time_pass(ctypes.c_void_p(plan), KERNEL_KINDS.index(kind),
                                   ctypes.c_void_p(observed_ptr), ctypes.c_void_p(estimate_ptr),
                                   int(reps), ctypes.byref(ms)))
    return ms.value


def rl_plan_get_pass_kernel(plan: int, kind: str):
    """(kernel names, threads per launch) of a pass kind as a profiler names them."""
    buf = ctypes.create_string_buffer(512)
    threads = ctypes.c_int64(0)
    _check(lib().rl_plan_get_pass_kernel(ctypes.c_void_p(plan), KERNEL_KINDS.index(kind), buf,
                                         ctypes.c_size_t(len(buf)), ctypes.byref(threads)))
    return buf.value.decode().split("|"), threads.value


def rl_probe_copy(src_ptr: int, dst_ptr: int, nbytes: int, stream: int = 0) -> None:
    _check(lib().rl_probe_copy(ctypes.c_void_p(src_ptr), ctypes.c_void_p(dst_ptr),
                               ctypes.c_size_t(nbytes), ctypes.c_void_p(stream or None)))


def rl_status_string(status: int) -> str:
    return lib().rl_status_string(int(status)).decode()


def rl_last_error() -> str:
    return lib().rl_last_error().decode(errors="replace")


# ---------------------------------------------------------------------------
# torch convenience layer
# ---------------------------------------------------------------------------

def _stream_of(device) -> int:
    import torch
    return int(torch.cuda.current_stream(device).cuda_stream)


def _check_volume(t, shape, device, name):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch.Tensor")
    if t.dtype != torch.float32:
        raise TypeError(f"{name} must be float32")
    if t.device.type != "cuda" or (device is not None and t.device != device):
        raise ValueError(f"{name} must live on {device}")
    if tuple(t.shape) != tuple(shape):
        raise ValueError(f"{name} has shape {tuple(t.shape)}, expected {tuple(shape)}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")


class Plan:
    """Richardson-Lucy plan for one volume shape and PSF (a float32 CUDA tensor [Z][Y][X]).

    `shape` is the volume's (Z, Y, X); None = the PSF's shape.  A smaller PSF is
    centred at floor(p/2) per axis.  boundary "periodic" (circular) or "zero"
    (linear convolution; the library pads the transform grid itself)."""

    def __init__(self, psf, boundary: str = "periodic", tile_x: int = 0, x_elems: int = 0,
                 yz_elems: int = 0, autotune: bool = False, precision: str = "fp32",
                 accel: str = "none", shape=None):
        bmap = {"periodic": RL_BOUNDARY_PERIODIC, "zero": RL_BOUNDARY_ZERO}
        if boundary not in bmap:
            raise ValueError("boundary must be 'periodic' or 'zero'")
        if psf.dim() != 3:
            raise ValueError("psf must be a 3-D tensor")
        _check_volume(psf, psf.shape, None, "psf")
        psf_shape = tuple(int(s) for s in psf.shape)
        self.shape = tuple(int(s) for s in shape) if shape is not None else psf_shape
        if len(self.shape) != 3:
            raise ValueError("shape must have three dimensions")
        self.device = psf.device
        if precision not in _PRECISIONS:
            raise ValueError(f"precision must be one of {sorted(_PRECISIONS)}")
        if accel not in _ACCELS:
            raise ValueError(f"accel must be one of {sorted(_ACCELS)}")
        self.accel = accel
        self.handle = rl_plan_create_ex(self.shape, psf.data_ptr(), bmap[boundary],
                                        precision=_PRECISIONS[precision],
                                        stream=_stream_of(self.device), tile_x=tile_x,
                                        x_elems=x_elems, yz_elems=yz_elems, autotune=autotune,
                                        accel=_ACCELS[accel],
                                        psf_shape=psf_shape if psf_shape != self.shape else (0, 0, 0))
        self.boundary = boundary

    def _bind_stream(self):
        rl_plan_set_stream(self.handle, _stream_of(self.device))

    def iterate(self, observed, estimate, n_iter: int) -> None:
        """Run n_iter iterations in place on `estimate` (asynchronous on torch's stream)."""
        self._live()
        _check_volume(observed, self.shape, self.device, "observed")
        _check_volume(estimate, self.shape, self.device, "estimate")
        self._bind_stream()
        rl_iterate(self.handle, observed.data_ptr(), estimate.data_ptr(), n_iter)

    def iterate_until(self, observed, estimate, max_iter: int, metric: str, threshold: float,
                      min_iter: int = 0, reference=None, fsc_bins: int = 0,
                      fsc_threshold: float = 0.0) -> None:
        """At most max_iter iterations, stopped on the device by `metric` ("loglik",
        "change", "fsc" (single-image FSC resolution; fsc_bins shells, crossing
        level fsc_threshold, 0 = defaults 64 and 1/7), or "psnr" / "ssim" against
        `reference`); results via stop() and flux()."""
        self._live()
        _check_volume(observed, self.shape, self.device, "observed")
        _check_volume(estimate, self.shape, self.device, "estimate")
        if metric not in _STOP_METRICS:
            raise ValueError(f"metric must be one of {sorted(_STOP_METRICS)}")
        ref_ptr = 0
        if metric in ("psnr", "ssim"):
            if reference is None:
                raise ValueError(f"{metric} needs a reference volume")
            _check_volume(reference, self.shape, self.device, "reference")
            ref_ptr = reference.data_ptr()
        self._bind_stream()
        rl_iterate_stop(self.handle, observed.data_ptr(), estimate.data_ptr(), max_iter,
                        _STOP_METRICS[metric], threshold, min_iter, ref_ptr, fsc_bins,
                        fsc_threshold)

    def iterate_until_fsc(self, observed, estimate, max_iter: int, threshold: float,
                          nbins: int = 64, fsc_threshold: float = 1.0 / 7.0, min_iter: int = 0):
        """iterate_until with the "fsc" rule: at most max_iter iterations, stopped on
        the device once the single-image FSC resolution of the estimate improves by
        less than `threshold` cycles per voxel between consecutive iterations.
        Returns (iterations done, resolution after each) (synchronises)."""
        self.iterate_until(observed, estimate, max_iter, "fsc", threshold, min_iter=min_iter,
                           fsc_bins=nbins, fsc_threshold=fsc_threshold)
        return self.stop()

    def stop(self):
        """(iterations done, metric history) of the last iterate_until call (synchronises)."""
        self._live()
        self._bind_stream()
        return rl_plan_get_stop(self.handle)

    def ssim(self, u, reference) -> float:
        """Mean SSIM (7x7x7 windows) of u against the reference (synchronises)."""
        self._live()
        _check_volume(u, self.shape, self.device, "u")
        _check_volume(reference, self.shape, self.device, "reference")
        self._bind_stream()
        return rl_ssim(self.handle, u.data_ptr(), reference.data_ptr())

    def fsc(self, a, b, nbins: int = 64, threshold: float = 1.0 / 7.0):
        """FSC curve of volumes a and b and the resolution crossing (synchronises)."""
        self._live()
        _check_volume(a, self.shape, self.device, "a")
        _check_volume(b, self.shape, self.device, "b")
        self._bind_stream()
        return rl_fsc(self.handle, a.data_ptr(), b.data_ptr(), nbins, threshold)

    def conv(self, x, out=None):
        """H x into `out` (new tensor if None)."""
        import torch
        self._live()
        _check_volume(x, self.shape, self.device, "x")
        if out is None:
            out = torch.empty_like(x)
        _check_volume(out, self.shape, self.device, "out")
        self._bind_stream()
        conv3d_fft(self.handle, x.data_ptr(), out.data_ptr())
        return out

    def flux(self) -> np.ndarray:
        """FP64 flux after each iteration of the last iterate() call (synchronises)."""
        self._live()
        self._bind_stream()
        return rl_plan_get_flux(self.handle)

    def alpha(self) -> np.ndarray:
        """Extrapolation weight of each iteration of the last iterate() call
        (plans with accel="biggs_andrews"; synchronises)."""
        self._live()
        self._bind_stream()
        return rl_plan_get_alpha(self.handle)

    def set_timing(self, enable: bool) -> None:
        self._live()
        rl_plan_set_timing(self.handle, enable)

    def timing(self) -> dict:
        self._live()
        self._bind_stream()
        return rl_plan_get_timing(self.handle)

    def info(self):
        self._live()
        return rl_plan_get_info(self.handle)

    def grid(self) -> tuple:
        """Transform grid (Z, Y, X): the volume's shape, or the padded grid of the zero boundary."""
        self._live()
        return rl_plan_get_grid(self.handle)

    def time_pass(self, kind: str, observed, estimate, reps: int = 20) -> float:
        """Steady-state ms per launch of a pass kind ('x_ratio', 'x_update', 'y', 'z_otf');
        overwrites `estimate` for 'x_update'."""
        self._live()
        _check_volume(observed, self.shape, self.device, "observed")
        _check_volume(estimate, self.shape, self.device, "estimate")
        self._bind_stream()
        return rl_plan_time_pass(self.handle, kind, observed.data_ptr(), estimate.data_ptr(), reps)

    def launch(self) -> dict:
        """Elements per thread and work-group widths in use (and whether tuned)."""
        self._live()
        return rl_plan_get_launch(self.handle)

    def pass_kernel(self, kind: str):
        """(kernel names, threads per launch) of a pass kind ('x_ratio', 'x_update',
        'y', 'z_otf') as a profiler's kernel trace names them."""
        self._live()
        return rl_plan_get_pass_kernel(self.handle, kind)

    def _live(self):
        if getattr(self, "handle", None) is None:
            raise RLError(RL_E_INVALID, "plan is closed")

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h is not None:
            self.handle = None
            rl_plan_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class BatchPlan:
    """Batched plan: volumes of uneven shape, each with its own PSF (float32 CUDA tensors)."""

    def __init__(self, psfs, autotune: bool = False, x_elems: int = 0, yz_elems: int = 0,
                 mode: str = "auto"):
        """mode: "graph" (per-pass kernels of each shape class in one graph per
        iteration), "auto" (the same) or "persistent" (one persistent kernel per
        iteration; switched off in the library, which refuses it with RL_E_UNSUPPORTED)."""
        if mode not in _BATCH_MODES:
            raise ValueError(f"mode must be one of {sorted(_BATCH_MODES)}")
        if len(psfs) == 0:
            raise ValueError("at least one volume")
        for i, h in enumerate(psfs):
            if h.dim() != 3:
                raise ValueError(f"psf {i} must be 3-D")
            _check_volume(h, h.shape, psfs[0].device, f"psf {i}")
        self.shapes = [tuple(int(v) for v in h.shape) for h in psfs]
        self.device = psfs[0].device
        self.handle = rl_plan_create_batch(self.shapes, [h.data_ptr() for h in psfs],
                                           stream=_stream_of(self.device), x_elems=x_elems,
                                           yz_elems=yz_elems, autotune=autotune,
                                           batch_mode=_BATCH_MODES[mode])

    def iterate(self, observed, estimates, n_iter: int) -> None:
        """n_iter iterations of every volume, in place on `estimates` (lists of tensors)."""
        self._live()
        if len(observed) != len(self.shapes) or len(estimates) != len(self.shapes):
            raise ValueError("one observed and one estimate tensor per volume")
        for i, shp in enumerate(self.shapes):
            _check_volume(observed[i], shp, self.device, f"observed {i}")
            _check_volume(estimates[i], shp, self.device, f"estimate {i}")
        rl_plan_set_stream(self.handle, _stream_of(self.device))
        rl_iterate_batch(self.handle, [t.data_ptr() for t in observed],
                         [t.data_ptr() for t in estimates], n_iter)

    def flux(self) -> np.ndarray:
        """(volumes, iterations) FP64 flux of the last iterate() call (synchronises)."""
        self._live()
        rl_plan_set_stream(self.handle, _stream_of(self.device))
        f = rl_plan_get_flux(self.handle)
        return f.reshape(len(self.shapes), -1)

    def launch(self) -> dict:
        self._live()
        return rl_plan_get_launch(self.handle)

    def mode(self) -> str:
        """"persistent" or "graph": how this plan runs its iterations."""
        self._live()
        return "persistent" if rl_plan_get_launch(self.handle)["batch_persistent"] else "graph"

    def _live(self):
        if getattr(self, "handle", None) is None:
            raise RLError(RL_E_INVALID, "plan is closed")

    def close(self) -> None:
        h = getattr(self, "handle", None)
        if h is not None:
            self.handle = None
            rl_plan_destroy(h)

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
