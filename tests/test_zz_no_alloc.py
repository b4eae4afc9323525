"""rl_iterate_noalloc (the iteration for callers that cannot allocate) against
rl_iterate, through the C ABI: the same kernels and partial sums, so the estimate
and the FP64 flux agree bit for bit.  Two calls in a row, the second on a smaller
volume, so the shared device scratch holds the first call's values when the
second one starts; then the limits, which are rejected before any device work."""

import ctypes
import sys

import numpy as np
import pytest

from paper_2510_14143_amd import rl, synth

pytestmark = pytest.mark.gpu


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    assert t.cuda.is_available()
    return t


def dev(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to("cuda:0")


def _both(torch, case, n_iter, autotune):
    """(u, flux) after rl_iterate and after rl_iterate_noalloc from the same start."""
    out = []
    with rl.Plan(dev(torch, case["psf"]), autotune=autotune) as p:
        d = dev(torch, case["d"])
        for fn in (rl.rl_iterate, rl.rl_iterate_noalloc):
            u = dev(torch, case["u0"])
            p._bind_stream()
            fn(p.handle, d.data_ptr(), u.data_ptr(), n_iter)
            flux = rl.rl_plan_get_flux(p.handle)
            out.append((u.cpu().numpy(), flux))
    return out


def test_noalloc_matches_rl_iterate_twice(torch):
    big = synth.make_config(1)            # 128x256x256, as benchmarked
    small = synth.small_case((16, 32, 64), seed=3)
    for name, case, n, tune in (("128x256x256", big, 40, True), ("16x32x64", small, 25, False)):
        say("noalloc vs rl_iterate", name, n, "iterations")
        (ua, fa), (ub, fb) = _both(torch, case, n, tune)
        assert fa.shape == fb.shape == (n,)
        assert np.array_equal(ua, ub), name
        assert np.array_equal(fa, fb), name
        total = float(case["d"].sum(dtype=np.float64))
        assert np.all(np.abs(fb - total) / total <= 1e-6), name


def test_noalloc_limits(torch):
    c = synth.small_case((16, 32, 64), seed=4)
    with rl.Plan(dev(torch, c["psf"])) as p:
        d = dev(torch, c["d"])
        u = dev(torch, c["u0"])
        keep = u.clone()
        L = rl.lib()
        # beyond the plan's flux capacity (128 for a new plan)
        st = L.rl_iterate_noalloc(ctypes.c_void_p(p.handle), ctypes.c_void_p(d.data_ptr()),
                                  ctypes.c_void_p(u.data_ptr()), 129)
        assert st == rl.RL_E_INVALID and "capacity" in rl.rl_last_error()
        assert L.rl_iterate_noalloc(ctypes.c_void_p(p.handle), ctypes.c_void_p(d.data_ptr()),
                                    ctypes.c_void_p(u.data_ptr()), -1) == rl.RL_E_INVALID
        p.set_timing(True)
        assert L.rl_iterate_noalloc(ctypes.c_void_p(p.handle), ctypes.c_void_p(d.data_ptr()),
                                    ctypes.c_void_p(u.data_ptr()), 2) == rl.RL_E_UNSUPPORTED
        p.set_timing(False)
        assert torch.equal(u, keep)  # nothing ran
    # the scratch bound: 2^20 partial values; the 256x512x512 plan has 16384 X
    # work-groups per iteration, so 65 iterations do not fit
    shape = synth.CONFIGS[2]["shape"]
    psf = dev(torch, synth.gaussian_psf(shape, synth.CONFIGS[2]["sigma"]))
    with rl.Plan(psf, x_elems=8) as p:
        d = torch.ones(shape, dtype=torch.float32, device="cuda:0")
        p.iterate(d, d.clone(), 65)  # grows the plan's flux capacity past 65
        st = rl.lib().rl_iterate_noalloc(ctypes.c_void_p(p.handle), ctypes.c_void_p(d.data_ptr()),
                                         ctypes.c_void_p(d.data_ptr()), 65)
        assert st == rl.RL_E_INVALID and "scratch" in rl.rl_last_error()
