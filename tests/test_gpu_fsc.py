"""Fourier shell correlation and the single-image split on the GPU against the FP64
oracle.

Bars: curve within 1e-5 of the oracle's (FP32 transforms, FP64 shell sums),
the resolution crossing within 1e-4 cycles per voxel, the split bit-exact."""

import sys

import numpy as np
import pytest

import oracle
from oracle import fsc_oracle as fo
from oracle import stop_oracle as so
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


@pytest.mark.parametrize("shape,nbins", [((16, 32, 64), 32), ((10, 20, 40), 16), ((24, 48, 96), 40),
                                         ((8, 16, 30), 8), ((1, 64, 64), 24)])
def test_fsc_matches_oracle(torch, shape, nbins):
    say("fsc", shape, nbins)
    rng = np.random.default_rng(90)
    a = synth.uniform_volume(shape, 91)
    b = (a + 0.5 * rng.normal(size=shape)).astype(np.float32)
    psf = synth.gaussian_psf(shape, (1.0, 1.0, 1.0))
    with rl.Plan(dev(torch, psf)) as p:
        curve, res = p.fsc(dev(torch, a), dev(torch, b), nbins)
        same, _ = p.fsc(dev(torch, a), dev(torch, a), nbins)
        neg, _ = p.fsc(dev(torch, a), dev(torch, -a), nbins)
    ref = fo.fsc(a, b, nbins)
    err = float(np.max(np.abs(curve - ref)))
    say("  max |d curve|", err, "res", res, fo.resolution(ref, nbins))
    assert err <= 1e-5
    assert abs(res - fo.resolution(ref, nbins)) <= 1e-4
    _, d1, _ = fo.fsc_sums(a, a, nbins)
    live = d1 > 1e-6 * d1.max()
    assert np.all(np.abs(same[live] - 1) <= 1e-6) and np.all(np.abs(neg[live] + 1) <= 1e-6)


def test_split_diagonal_exact(torch):
    u = synth.uniform_volume((6, 10, 14), 92)
    a, b = rl.split_diagonal(dev(torch, u))
    ra, rb = fo.split_diagonal(u)
    assert np.array_equal(a.cpu().numpy(), ra) and np.array_equal(b.cpu().numpy(), rb)


def test_single_image_fsc_of_a_deconvolution(torch):
    shape = (32, 64, 64)
    say("single-image fsc")
    c = synth.small_case(shape, seed=93)
    with rl.Plan(dev(torch, c["psf"])) as p:
        u = dev(torch, c["u0"])
        p.iterate(dev(torch, c["d"]), u, 10)
        est = u.cpu().numpy()
        a, b = rl.split_diagonal(u)
    half = tuple(n // 2 for n in shape)
    with rl.Plan(dev(torch, synth.gaussian_psf(half, (1.0, 1.0, 1.0)))) as q:
        curve, res = q.fsc(a, b, 16)
    ra, rb = fo.split_diagonal(est)
    ref = fo.fsc(ra, rb, 16)
    assert np.max(np.abs(curve - ref)) <= 1e-5
    assert abs(res - fo.resolution(ref, 16)) <= 1e-4


def test_fsc_errors(torch):
    shape = (8, 16, 32)
    x = dev(torch, synth.uniform_volume(shape, 94))
    psf = dev(torch, synth.gaussian_psf(shape, (1.0, 1.0, 1.0)))
    with rl.Plan(psf) as p:
        for nb in (1, 1025):
            with pytest.raises(rl.RLError) as ei:
                p.fsc(x, x, nb)
            assert ei.value.status == rl.RL_E_INVALID
    with rl.Plan(dev(torch, synth.gaussian_psf((3, 3, 3), (1.0, 1.0, 1.0))), shape=shape,
                 boundary="zero") as p:
        with pytest.raises(rl.RLError) as ei:
            p.fsc(x, x)
        assert ei.value.status == rl.RL_E_UNSUPPORTED
    with pytest.raises(rl.RLError):
        rl.split_diagonal(dev(torch, np.ones((3, 4, 4))))


def test_fsc_guided_stop_matches_oracle(torch):
    c = synth.make_config(0)
    say("fsc-guided stop")
    nb = 16
    _, _, full = so.rl_stop(c["d"], c["psf"], c["u0"], 20, "fsc", -1e300, nbins=nb)
    delta = np.diff(full)                       # delta[j]: after iteration j + 2
    # a threshold halfway between two well-separated consecutive improvements
    gaps = [(abs(delta[j] - delta[j + 1]), j) for j in range(2, len(delta) - 1)
            if delta[j + 1] < delta[j]]
    _, j = max(gaps)
    tau = 0.5 * (delta[j] + delta[j + 1])
    ref_u, ref_n, ref_hist = so.rl_stop(c["d"], c["psf"], c["u0"], 20, "fsc", tau, nbins=nb)
    with rl.Plan(dev(torch, c["psf"])) as p:
        u = dev(torch, c["u0"])
        n, hist = p.iterate_until_fsc(dev(torch, c["d"]), u, 20, tau, nbins=nb)
        got = u.cpu().numpy()
    say("  oracle n", ref_n, "gpu n", n, "tau", tau)
    assert n == ref_n
    assert np.max(np.abs(hist - ref_hist)) <= 1e-4
    assert np.max(np.abs(got - ref_u)) / np.max(np.abs(ref_u)) <= 1e-4


def test_full_size_single_image_fsc_as_benchmarked(torch):
    # the benchmark's FSC: the 128x256x256 observed volume split into its two
    # diagonal 64x128x128 halves, 64 shells, against the oracle
    c = synth.make_config(1)
    say("full-size single-image fsc", c["shape"])
    d = dev(torch, c["d"])
    a, b = rl.split_diagonal(d)
    half = tuple(n // 2 for n in c["shape"])
    with rl.Plan(dev(torch, synth.gaussian_psf(half, (1.0, 1.0, 1.0)))) as q:
        curve, res = q.fsc(a, b, 64)
    ra, rb = fo.split_diagonal(c["d"])
    ref = fo.fsc(ra, rb, 64)
    err = float(np.max(np.abs(curve - ref)))
    say("  max |d curve|", err, "resolution", res, fo.resolution(ref, 64))
    assert err <= 1e-5
    assert abs(res - fo.resolution(ref, 64)) <= 1e-4


def test_fsc_stop_rule_errors(torch):
    # FSC-guided stopping through the C ABI: bad shell counts and thresholds are
    # rejected before any device work, odd dimensions and the zero boundary are not
    # supported
    shape = (8, 16, 32)
    d = dev(torch, synth.uniform_volume(shape, 95) + 1.0)
    psf = dev(torch, synth.gaussian_psf(shape, (1.0, 1.0, 1.0)))
    with rl.Plan(psf) as p:
        u = d.clone()
        for nb in (1, 1025, -3):
            with pytest.raises(rl.RLError) as ei:
                p.iterate_until(d, u, 3, "fsc", 0.0, fsc_bins=nb)
            assert ei.value.status == rl.RL_E_INVALID
        with pytest.raises(rl.RLError) as ei:
            p.iterate_until(d, u, 3, "fsc", 0.0, fsc_threshold=float("nan"))
        assert ei.value.status == rl.RL_E_INVALID
        assert torch.equal(u, d)  # nothing ran
    odd = (8, 16, 18)  # the half-size volume would have 9 columns (odd nx is not supported)
    with rl.Plan(dev(torch, synth.gaussian_psf(odd, (1.0, 1.0, 1.0)))) as p:
        dd = dev(torch, synth.uniform_volume(odd, 96) + 1.0)
        with pytest.raises(rl.RLError) as ei:
            p.iterate_until(dd, dd.clone(), 3, "fsc", 0.0)
        assert ei.value.status == rl.RL_E_UNSUPPORTED
    with rl.Plan(dev(torch, synth.gaussian_psf((3, 3, 3), (1.0, 1.0, 1.0))), shape=shape,
                 boundary="zero") as p:
        with pytest.raises(rl.RLError) as ei:
            p.iterate_until(d, d.clone(), 3, "fsc", 0.0)
        assert ei.value.status == rl.RL_E_UNSUPPORTED


def test_fsc_stop_history_full_size(torch):
    # the benchmark's 128x256x256 volume: the device rule's resolution history over 3
    # iterations (it never fires) against the stop oracle's
    c = synth.make_config(1)
    say("full-size fsc-guided stop history", c["shape"])
    n = 3
    ref_u, ref_n, ref_hist = so.rl_stop(c["d"], c["psf"], c["u0"], n, "fsc", -1e300, nbins=64)
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        u = dev(torch, c["u0"])
        n_done, hist = p.iterate_until_fsc(dev(torch, c["d"]), u, n, -1e300, nbins=64)
        got = u.cpu().numpy()
    say("  gpu", hist, "oracle", ref_hist)
    assert n_done == ref_n == n
    assert np.max(np.abs(hist - ref_hist)) <= 1e-4
    assert oracle.rel_l2(got, ref_u) <= 1e-5
