"""Transform lengths with radix-5, radix-7 and several odd stages (o * 2^a, o in
{1, 3, 5, 7, 9, 15}) on the GPU against the FP64 oracle.

Bars as for the other lengths: convolution within 1e-5 relative L2,
Richardson-Lucy within 1e-4 after 20 iterations, flux within 1e-5."""

import sys

import numpy as np
import pytest

import oracle
from oracle import boundary_oracle as bo
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


def rand_psf(shape, seed):
    h = np.random.default_rng(seed).uniform(0, 1, size=shape) ** 4
    h[tuple(n // 3 for n in shape)] += 3.0
    return h.astype(np.float32)


SHAPES = [(10, 20, 40), (7, 28, 56), (9, 18, 36), (15, 30, 60), (5, 40, 80), (30, 60, 30),
          (14, 36, 72), (20, 80, 160), (30, 240, 320), (1, 5, 10), (3, 7, 14)]


@pytest.mark.parametrize("shape", SHAPES)
def test_conv_odd_radices(torch, shape):
    say("conv", shape)
    x = synth.uniform_volume(shape, 400)
    psf = rand_psf(shape, 401)
    with rl.Plan(dev(torch, psf)) as p:
        cfg = p.launch()
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.conv3d(x, psf))
    say("  relL2", err, cfg)
    assert err <= 1e-5


@pytest.mark.parametrize("x_elems,yz_elems", [(10, 10), (10, 20), (20, 10)])
def test_conv_odd_radix_element_counts(torch, x_elems, yz_elems):
    shape = (20, 40, 80)
    say("conv elems", x_elems, yz_elems)
    x = synth.uniform_volume(shape, 402)
    psf = rand_psf(shape, 403)
    with rl.Plan(dev(torch, psf), x_elems=x_elems, yz_elems=yz_elems) as p:
        cfg = p.launch()
        got = p.conv(dev(torch, x)).cpu().numpy()
    assert cfg["x_elems"] == x_elems and cfg["y_elems"] == yz_elems
    assert oracle.rel_l2(got, oracle.conv3d(x, psf)) <= 1e-5


@pytest.mark.parametrize("shape", [(20, 40, 80), (14, 28, 56), (30, 60, 120)])
def test_rl_odd_radices(torch, shape):
    say("rl", shape)
    c = synth.small_case(shape, sigma_xyz=(1.5, 1.5, 2.5), seed=71)
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        u = dev(torch, c["u0"])
        p.iterate(dev(torch, c["d"]), u, 20)
        got = u.cpu().numpy()
        flux = p.flux()
    ref, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], 20)
    err = oracle.rel_l2(got, ref)
    say("  relL2", err)
    assert err <= 1e-4
    total = float(c["d"].sum(dtype=np.float64))
    assert np.all(np.abs(flux - total) / total <= 1e-5)


def test_zero_boundary_uses_odd_lengths(torch):
    # 148 planes pad to 160 = 5 * 32, 264 rows and columns to 320 = 5 * 64
    shape, pshape = (128, 256, 256), (41, 17, 17)
    say("zero grid", shape)
    h = synth.gaussian_psf(pshape, (2.0, 2.0, 5.0))
    with rl.Plan(dev(torch, h), shape=shape, boundary="zero") as p:
        assert p.grid() == (160, 320, 320)
        x = synth.uniform_volume(shape, 404)
        got = p.conv(dev(torch, x)).cpu().numpy()
    pts = [(0, 0, 0), (127, 255, 255), (64, 3, 250), (5, 128, 1), (100, 200, 17), (127, 0, 128)]
    ref = bo.conv_zero_at(x, h, pts)
    for pt, r in zip(pts, ref):
        assert abs(got[pt] - r) <= 1e-5 * max(1.0, abs(r)), (pt, got[pt], r)


def test_small_psf_with_odd_lengths(torch):
    shape, pshape = (15, 40, 60), (5, 9, 7)
    x = synth.uniform_volume(shape, 405)
    h = rand_psf(pshape, 406)
    with rl.Plan(dev(torch, h), shape=shape) as p:
        got = p.conv(dev(torch, x)).cpu().numpy()
    assert oracle.rel_l2(got, bo.conv_periodic(x, h)) <= 1e-5


@pytest.mark.parametrize("shape", [(2, 1024, 2048), (1024, 2, 2048), (1, 4, 3072), (3, 960, 8),
                                   (2, 2, 2560)])
def test_conv_maximum_lengths_sampled(torch, shape):
    # the longest transforms per axis (nx 2048, 3072 = 24 * 128, 2560 = 20 * 128 split over
    # 64 threads; ny, nz 1024 and 960 = 15 * 64), sampled voxels by the direct sum
    say("max conv", shape)
    x = synth.uniform_volume(shape, 407)
    rng = np.random.default_rng(408)
    psf = np.zeros(shape, np.float32)
    for _ in range(40):  # a sparse, asymmetric PSF keeps the direct sums cheap
        psf[tuple(int(rng.integers(0, n)) for n in shape)] += float(rng.uniform(0.1, 1.0))
    with rl.Plan(dev(torch, psf)) as p:
        got = p.conv(dev(torch, x)).cpu().numpy()
    pts = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(8)]
    pts += [(0, 0, 0), tuple(n - 1 for n in shape)]
    ref = oracle.conv_direct_at(x, psf, pts)
    g = np.array([got[q] for q in pts])
    assert np.max(np.abs(g - ref) / np.abs(ref)) <= 1e-5


def test_batch_with_odd_radix_shapes(torch):
    shapes = [(10, 20, 40), (7, 14, 28), (10, 20, 40), (9, 18, 36)]
    say("batch odd radices")
    cases = [synth.small_case(s, sigma_xyz=(1.2, 1.2, 2.0), seed=409 + k) for k, s in enumerate(shapes)]
    with rl.BatchPlan([dev(torch, c["psf"]) for c in cases]) as b:
        ds = [dev(torch, c["d"]) for c in cases]
        us = [dev(torch, c["u0"]) for c in cases]
        b.iterate(ds, us, 12)
        got = [u.cpu().numpy() for u in us]
    for c, g in zip(cases, got):
        ref, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], 12)
        assert oracle.rel_l2(g, ref) <= 1e-4


# Y and Z lengths whose odd part has a repeated prime (27, 25, 45, 135) or which
# are longer than 1024: their elements-per-thread count carries every odd prime
# once and the thread count per pencil the rest (2160 = 16 * 135: 30 elements on
# 72 threads)
LONG_SHAPES = [(27, 8, 8), (4, 25, 16), (45, 18, 8), (2, 270, 16), (4, 2160, 8), (1080, 2, 8),
               (2048, 4, 8), (3, 4096, 4)]


@pytest.mark.parametrize("shape", LONG_SHAPES)
def test_conv_repeated_odd_primes_and_long_pencils(torch, shape):
    say("conv long/odd", shape)
    x = synth.uniform_volume(shape, 410)
    psf = rand_psf(shape, 411)
    with rl.Plan(dev(torch, psf)) as p:
        cfg = p.launch()
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, oracle.conv3d(x, psf))
    say("  relL2", err, cfg)
    assert err <= 1e-5


@pytest.mark.parametrize("shape", [(6, 270, 32), (4, 2160, 16)])
def test_rl_long_pencils(torch, shape):
    say("rl long", shape)
    c = synth.small_case(shape, sigma_xyz=(1.5, 2.5, 2.0), seed=72)
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        u = dev(torch, c["u0"])
        p.iterate(dev(torch, c["d"]), u, 10)
        got = u.cpu().numpy()
        flux = p.flux()
    ref, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], 10)
    err = oracle.rel_l2(got, ref)
    say("  relL2", err)
    assert err <= 1e-4
    total = float(c["d"].sum(dtype=np.float64))
    assert np.all(np.abs(flux - total) / total <= 1e-5)
