"""The kernels compiled for fixed transform lengths, each against the FP64 oracle
and each checked to be the kernel that ran (by the name the plan reports for
its pass):

* pencils of 128, 256 and 512 points with 16 elements per thread (FP32 and both
  split precisions),
* pencils of 32 ... 512 points with 8 elements per thread (up to 1024-thread
  work-groups),
* the 3 * 2^a pencils and X rows of the batched volumes (pencils of 24, 48 and
  96 points with 6 elements, of 48, 96 and 192 with 12; rows of 24, 48 and 96
  points with 6),
* the 2160-point pencils of the paper's stack (30 elements per thread),
* the fused X passes of 1280-point rows (nx = 2560, 20 elements per thread).

Bars as for the other lengths: convolution within 1e-5 relative L2 (split: the
split-precision bars), Richardson-Lucy within 1e-4 (split: 5e-4), flux within
1e-5 of the observed total."""

import sys

import numpy as np
import pytest

import oracle
from paper_2510_14143_amd import rl, synth

pytestmark = pytest.mark.gpu

CONV_TOL = {"fp32": 1e-5, "split_bf16": 1e-4, "split_fp16": 1e-5}
RL_TOL = {"fp32": 1e-4, "split_bf16": 5e-4, "split_fp16": 5e-4}


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


def rand_psf(shape, seed):
    h = np.random.default_rng(seed).uniform(0, 1, size=shape) ** 4
    h[tuple(n // 3 for n in shape)] += 3.0
    return h.astype(np.float32)


def check_rl(torch, plan, c, n_iter, tol):
    d, u = dev(torch, c["d"]), dev(torch, c["u0"])
    plan.iterate(d, u, n_iter)
    flux = plan.flux()
    ref, ref_flux, _ = oracle.rl(c["d"], c["psf"], c["u0"], n_iter)
    err = oracle.rel_l2(u.cpu().numpy(), ref)
    total = float(c["d"].sum(dtype=np.float64))
    say("  RL relL2", err, "flux", float(np.max(np.abs(flux - ref_flux) / ref_flux)))
    assert err <= tol
    assert np.all(np.abs(flux - total) / total <= 1e-5)


# (shape, Y kernel, Z kernel) with 16 elements per thread on Y and Z
PENCIL_CASES = [((128, 512, 16), 512, 128), ((256, 128, 16), 128, 256), ((128, 256, 32), 256, 128)]


@pytest.mark.parametrize("precision", ["fp32", "split_bf16", "split_fp16"])
@pytest.mark.parametrize("shape,ly,lz", PENCIL_CASES)
def test_compiled_pencils(torch, precision, shape, ly, lz):
    say("compiled pencils", precision, shape)
    prec = {"fp32": 0, "split_bf16": 1, "split_fp16": 2}[precision]
    x = synth.uniform_volume(shape, 500)
    psf = rand_psf(shape, 501)
    with rl.Plan(dev(torch, psf), yz_elems=16, precision=precision) as p:
        ny, _ = p.pass_kernel("y")
        nz, _ = p.pass_kernel("z_otf")
        say("  kernels", ny, nz)
        assert ny == [f"k_pencil_ct<16, 0, {prec}, {ly}>", f"k_pencil_ct<16, 1, {prec}, {ly}>"]
        assert nz == [f"k_pencil_ct<16, 2, {prec}, {lz}>", f"k_pencil_ct<16, 3, {prec}, {lz}>"]
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.conv3d(x, psf))
    say("  conv relL2", err)
    assert err <= CONV_TOL[precision]
    c = synth.small_case(shape, seed=502, density=4.0)
    with rl.Plan(dev(torch, c["psf"]), yz_elems=16, precision=precision) as p:
        check_rl(torch, p, c, 5, RL_TOL[precision])


# (shape, elements per thread on Y and Z, Y length, Z length)
BATCH_PENCIL_CASES = [((24, 48, 16), 6, 48, 24), ((48, 96, 16), 6, 96, 48),
                      ((48, 96, 16), 12, 96, 48), ((96, 192, 16), 12, 192, 96),
                      ((64, 128, 16), 8, 128, 64), ((32, 512, 16), 8, 512, 32),
                      ((256, 256, 8), 8, 256, 256)]


@pytest.mark.parametrize("shape,e,ly,lz", BATCH_PENCIL_CASES)
def test_compiled_batch_pencils(torch, shape, e, ly, lz):
    say("compiled pencils", shape, e)
    x = synth.uniform_volume(shape, 530)
    psf = rand_psf(shape, 531)
    with rl.Plan(dev(torch, psf), yz_elems=e) as p:
        ny, _ = p.pass_kernel("y")
        nz, _ = p.pass_kernel("z_otf")
        say("  kernels", ny, nz)
        assert ny == [f"k_pencil_ct<{e}, 0, 0, {ly}>", f"k_pencil_ct<{e}, 1, 0, {ly}>"]
        assert nz == [f"k_pencil_ct<{e}, 2, 0, {lz}>", f"k_pencil_ct<{e}, 3, 0, {lz}>"]
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.conv3d(x, psf))
    say("  conv relL2", err)
    assert err <= CONV_TOL["fp32"]
    c = synth.small_case(shape, seed=532, density=4.0)
    with rl.Plan(dev(torch, c["psf"]), yz_elems=e) as p:
        check_rl(torch, p, c, 5, RL_TOL["fp32"])


@pytest.mark.parametrize("nx", [48, 96, 192])
def test_compiled_batch_rows(torch, nx):
    shape = (6, 8, nx)
    say("compiled rows", shape)
    c = synth.small_case(shape, seed=540 + nx, density=16.0)
    with rl.Plan(dev(torch, c["psf"]), x_elems=6) as p:
        r, _ = p.pass_kernel("x_ratio")
        u, _ = p.pass_kernel("x_update")
        say("  kernels", r, u)
        assert r == [f"k_xrow<6, 2, 0, {nx // 2}>"] and u == [f"k_xrow<6, 3, 0, {nx // 2}>"]
        check_rl(torch, p, c, 5, RL_TOL["fp32"])


def test_compiled_2160_point_pencils(torch):
    # the paper stack's Y length: 30 elements on 72 threads per pencil, 8 lanes
    shape = (2, 2160, 16)
    say("compiled 2160-point pencils", shape)
    x = synth.uniform_volume(shape, 510)
    psf = rand_psf(shape, 511)
    with rl.Plan(dev(torch, psf)) as p:
        names, threads = p.pass_kernel("y")
        launch = p.launch()
        say("  kernels", names, threads, launch)
        assert names == ["k_pencil_ct<30, 0, 0, 2160>", "k_pencil_ct<30, 1, 0, 2160>"]
        assert launch["y_elems"] == 30 and launch["y_lanes"] == 8
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.conv3d(x, psf))
    say("  conv relL2", err)
    assert err <= CONV_TOL["fp32"]
    c = synth.small_case(shape, seed=512, density=8.0)
    with rl.Plan(dev(torch, c["psf"])) as p:
        check_rl(torch, p, c, 5, RL_TOL["fp32"])


def test_compiled_1280_point_rows(torch):
    # the paper stack's X length: rows of 2560 samples, 1280-point complex rows
    shape = (2, 12, 2560)
    say("compiled 1280-point rows", shape)
    c = synth.small_case(shape, seed=520, density=8.0)
    with rl.Plan(dev(torch, c["psf"]), x_elems=20) as p:
        r, _ = p.pass_kernel("x_ratio")
        u, _ = p.pass_kernel("x_update")
        say("  kernels", r, u)
        assert r == ["k_xrow<20, 2, 0, 1280>"] and u == ["k_xrow<20, 3, 0, 1280>"]
        check_rl(torch, p, c, 5, RL_TOL["fp32"])
