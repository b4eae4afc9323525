"""Split-precision form: radix-16 butterflies as DFT matrix products on MFMA with
BF16 or FP16 hi/lo operands, against the FP64 oracle.

Bars: Richardson-Lucy after 10 and 50 iterations within 5e-4 relative L2 of the
oracle (both splits; the plain FP32 form within 1e-4).  A single convolution:
BF16 split within 1e-4 (its operands carry ~16 significant bits), FP16 split
within 1e-5 (~22 bits).  At the full 512x512x256 size the oracle's values come
from tests/golden/rl_512x512x256_samples.txt (written by the script beside it,
which calls only the oracle), compared at its sample voxels."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14143_amd import rl, synth

pytestmark = pytest.mark.gpu

SPLITS = ["split_bf16", "split_fp16"]
CONV_TOL = {"split_bf16": 1e-4, "split_fp16": 1e-5}
RL_TOL = 5e-4


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


@pytest.mark.parametrize("precision", SPLITS)
@pytest.mark.parametrize("shape", [(16, 32, 64), (32, 64, 64), (16, 16, 256), (24, 48, 96)])
def test_split_conv(torch, precision, shape):
    say("split conv", precision, shape)
    x = synth.uniform_volume(shape, 200)
    rng = np.random.default_rng(3)
    psf = (rng.uniform(0, 1, size=shape) ** 4).astype(np.float32)
    psf[tuple(s // 3 for s in shape)] += 5.0
    ref = oracle.conv3d(x, psf)
    with rl.Plan(dev(torch, psf), precision=precision) as p:
        cfg = p.launch()
        got = p.conv(dev(torch, x)).cpu().numpy()
    err = oracle.rel_l2(got, ref)
    say("  relL2", err, cfg)
    assert err <= CONV_TOL[precision]


@pytest.mark.parametrize("precision", SPLITS)
@pytest.mark.parametrize("shape", [(16, 32, 64), (32, 64, 64), (16, 16, 256)])
def test_split_conv_mfma_x_passes(torch, precision, shape):
    # x_elems = 16: the fused X passes run their radix-16 stages on MFMA too
    say("split conv, MFMA X passes", precision, shape)
    x = synth.uniform_volume(shape, 202)
    rng = np.random.default_rng(4)
    psf = (rng.uniform(0, 1, size=shape) ** 4).astype(np.float32)
    psf[tuple(s // 3 for s in shape)] += 5.0
    ref = oracle.conv3d(x, psf)
    with rl.Plan(dev(torch, psf), precision=precision, x_elems=16) as p:
        cfg = p.launch()
        got = p.conv(dev(torch, x)).cpu().numpy()
    assert cfg["x_elems"] == 16
    err = oracle.rel_l2(got, ref)
    say("  relL2", err, cfg)
    assert err <= CONV_TOL[precision]


@pytest.mark.parametrize("precision", SPLITS)
def test_split_rl_mfma_x_passes(torch, precision):
    c = synth.make_config(0)
    say("split rl, MFMA X passes", precision)
    with rl.Plan(dev(torch, c["psf"]), precision=precision, x_elems=16) as p:
        u = dev(torch, c["u0"])
        p.iterate(dev(torch, c["d"]), u, 10)
        got = u.cpu().numpy()
    ref = oracle.rl(c["d"], c["psf"], c["u0"], 10)[0]
    err = oracle.rel_l2(got, ref)
    say("  relL2", err)
    assert err <= RL_TOL


@pytest.mark.parametrize("precision", SPLITS)
def test_split_conv_gaussian_psf_tail(torch, precision):
    # a Gaussian PSF over the whole grid has FP32 values far below 2^-100 in its
    # tail: the FP16 per-DFT scale must stay finite there
    shape = (32, 64, 64)
    say("split conv gaussian", precision)
    x = synth.uniform_volume(shape, 201)
    psf = synth.gaussian_psf(shape, (1.5, 1.5, 3.0))
    ref = oracle.conv3d(x, psf)
    with rl.Plan(dev(torch, psf), precision=precision) as p:
        got = p.conv(dev(torch, x)).cpu().numpy()
    assert np.all(np.isfinite(got))
    assert oracle.rel_l2(got, ref) <= CONV_TOL[precision]


@pytest.mark.parametrize("precision", SPLITS)
def test_split_rl_10_and_50(torch, precision):
    c = synth.make_config(0)
    say("split rl config0", precision)
    with rl.Plan(dev(torch, c["psf"]), precision=precision) as p:
        d = dev(torch, c["d"])
        u = dev(torch, c["u0"])
        p.iterate(d, u, 10)
        u10 = u.cpu().numpy()
        p.iterate(d, u, 40)
        u50 = u.cpu().numpy()
        flux = p.flux()
    r10, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], 10)
    r50, f50, _ = oracle.rl(c["d"], c["psf"], c["u0"], 50)
    e10, e50 = oracle.rel_l2(u10, r10), oracle.rel_l2(u50, r50)
    say("  relL2 at 10:", e10, " at 50:", e50)
    assert e10 <= RL_TOL and e50 <= RL_TOL
    total = float(c["d"].sum(dtype=np.float64))
    assert np.all(np.abs(flux - total) / total <= 1e-5)
    assert np.all(u50 >= 0)


@pytest.mark.parametrize("precision", SPLITS)
def test_split_rl_larger_volume(torch, precision):
    shape = (64, 128, 128)
    say("split rl", shape, precision)
    c = synth.small_case(shape, sigma_xyz=(2.0, 2.0, 4.0), seed=31)
    with rl.Plan(dev(torch, c["psf"]), precision=precision) as p:
        u = dev(torch, c["u0"])
        p.iterate(dev(torch, c["d"]), u, 10)
        got = u.cpu().numpy()
    ref, _, _ = oracle.rl(c["d"], c["psf"], c["u0"], 10)
    err = oracle.rel_l2(got, ref)
    say("  relL2 at 10:", err)
    assert err <= RL_TOL


GOLDEN_512 = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                          "rl_512x512x256_samples.txt")


@pytest.fixture(scope="module")
def organoid():
    return synth.make_config(2)


@pytest.mark.parametrize("precision,tol", [("fp32", 1e-4), ("split_bf16", RL_TOL),
                                           ("split_fp16", RL_TOL)])
def test_full_size_512_against_oracle_samples(torch, organoid, precision, tol):
    # the 512x512x256 workload as the benchmark runs it (FP32 autotuned, the splits
    # with their default shapes); relative L2 over the oracle's sample voxels
    a = np.loadtxt(GOLDEN_512, comments="#")
    pts, ref = a[:, :3].astype(np.int64), {10: a[:, 3], 50: a[:, 4]}
    c = organoid
    assert tuple(c["shape"]) == (256, 512, 512)
    say("full-size 512x512x256 vs oracle samples", precision)
    idx = torch.from_numpy(pts).to("cuda:0")
    with rl.Plan(dev(torch, c["psf"]), precision=precision,
                 autotune=precision == "fp32") as p:
        d, u = dev(torch, c["d"]), dev(torch, c["u0"])
        got = {}
        done = 0
        for n in (10, 50):
            p.iterate(d, u, n - done)
            done = n
            got[n] = u[idx[:, 0], idx[:, 1], idx[:, 2]].double().cpu().numpy()
    for n in (10, 50):
        err = float(np.linalg.norm(got[n] - ref[n]) / np.linalg.norm(ref[n]))
        say(f"  after {n}: relative L2 over {len(pts)} voxels {err:.3e}")
        assert err <= tol
