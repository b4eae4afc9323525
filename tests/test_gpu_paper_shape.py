"""The paper's own stack shape, 30x2160x2560 (Z, Y, X; §4.3, paragraph "Dataset
description"), on the GPU: 2160 = 16 * 135 runs as a pencil of 30 elements on 72
threads.  Plans with both boundaries; one convolution at sampled voxels against
the oracle's direct sum; two Richardson-Lucy iterations against the FP64 oracle's
stored estimate at sampled voxels (tests/golden/make_rl_paper_shape_samples.py)."""

import os
import sys

import numpy as np
import pytest

import oracle
from paper_2510_14143_amd import rl, synth

pytestmark = pytest.mark.gpu

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden",
                      "rl_paper_shape_samples.txt")


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


def test_plans_for_the_paper_shape(torch):
    shape = synth.PAPER_SHAPE
    psf = torch.zeros(shape, dtype=torch.float32, device="cuda:0")
    psf[tuple(n // 2 for n in shape)] = 1.0
    with rl.Plan(psf) as p:
        assert p.grid() == shape
        say("periodic launch", p.launch())
    small = dev(torch, synth.gaussian_psf((15, 31, 31), synth.PAPER_SIGMA))
    with rl.Plan(small, shape=shape, boundary="zero") as p:
        g = p.grid()
        say("zero-boundary grid", g)
        assert all(gi >= n + pn // 2 for gi, n, pn in zip(g, shape, (15, 31, 31)))


def test_conv_paper_shape_sampled(torch):
    shape = synth.PAPER_SHAPE
    say("conv", shape)
    x = synth.uniform_volume(shape, 2161)
    rng = np.random.default_rng(2162)
    psf = np.zeros(shape, np.float32)
    for _ in range(40):  # a sparse, asymmetric PSF keeps the direct sums cheap
        psf[tuple(int(rng.integers(0, n)) for n in shape)] += float(rng.uniform(0.1, 1.0))
    with rl.Plan(dev(torch, psf)) as p:
        got = p.conv(dev(torch, x)).cpu().numpy()
    pts = [tuple(int(rng.integers(0, n)) for n in shape) for _ in range(3)]
    pts += [(0, 0, 0), tuple(n - 1 for n in shape)]
    ref = oracle.conv_direct_at(x, psf, pts)
    g = np.array([got[q] for q in pts])
    err = float(np.max(np.abs(g - ref) / np.abs(ref)))
    say("  max rel error", err)
    assert err <= 1e-5


def test_rl_paper_shape_vs_oracle_samples(torch):
    c = synth.make_paper_shape()
    a = np.loadtxt(GOLDEN, comments="#")
    with open(GOLDEN) as f:
        ref_flux = [float(t) for t in next(ln for ln in f if ln.startswith("# flux:")).split()[2:]]
    pts = a[:, :3].astype(np.int64)
    say("rl 2 iterations", c["shape"])
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        d = dev(torch, c["d"])
        u = dev(torch, c["u0"])
        p.iterate(d, u, 1)
        u1 = u.cpu().numpy().astype(np.float64)
        f1 = p.flux()
        p.iterate(d, u, 1)
        u2 = u.cpu().numpy().astype(np.float64)
        f2 = p.flux()
        say("  launch", p.launch())
    for k, got, ref, fl, rf in ((1, u1, a[:, 3], f1, ref_flux[0]), (2, u2, a[:, 4], f2, ref_flux[1])):
        g = got[tuple(pts.T)]
        err = float(np.linalg.norm(g - ref) / np.linalg.norm(ref))
        say(f"  {k} iteration(s): relL2 over {len(ref)} samples {err:.3e}")
        assert err <= 1e-5
        assert abs(fl[-1] - rf) / rf <= 1e-6
