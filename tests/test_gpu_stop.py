"""Metric-guided stopping on the GPU against the FP64 stopping oracle.

The threshold of each case is placed halfway between two consecutive
improvements of the oracle's own metric history, so the stop iteration is
unambiguous; the GPU must stop at the same iteration, with the estimate within
1e-4 relative L2 of the oracle's, and report the metric history within
1e-6 relative (log-likelihood, change) or 1e-3 dB (PSNR)."""

import sys

import numpy as np
import pytest

import oracle
from oracle import boundary_oracle as bo
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


def _threshold(metric, hist, s):
    """Threshold between the checks before and at position s of the history."""
    if metric == "loglik":
        delta = np.diff(hist) / np.abs(hist[1:])   # delta[j]: check at iteration j + 1
        return 0.5 * (delta[s - 2] + delta[s - 1])
    if metric == "change":
        return 0.5 * (hist[s - 2] + hist[s - 1])
    delta = np.diff(hist)                           # delta[j]: after iteration j + 2
    return 0.5 * (delta[s - 3] + delta[s - 2])


@pytest.mark.parametrize("metric,s", [("loglik", 8), ("change", 9), ("psnr", 6)])
def test_stop_matches_oracle(torch, metric, s):
    c = synth.make_config(0)
    say("stop", metric)
    truth = c["truth"].astype(np.float32)
    _, _, full = so.rl_stop(c["d"], c["psf"], c["u0"], 25, metric, -1e300, reference=truth)
    tau = _threshold(metric, full, s)
    ref_u, ref_n, ref_hist = so.rl_stop(c["d"], c["psf"], c["u0"], 25, metric, tau, reference=truth)
    with rl.Plan(dev(torch, c["psf"])) as p:
        u = dev(torch, c["u0"])
        p.iterate_until(dev(torch, c["d"]), u, 25, metric, tau,
                        reference=dev(torch, truth) if metric == "psnr" else None)
        n, hist = p.stop()
        flux = p.flux()
        got = u.cpu().numpy()
    say("  oracle n", ref_n, "gpu n", n, "tau", tau)
    assert n == ref_n
    assert len(hist) == len(ref_hist)
    if metric == "psnr":
        assert np.max(np.abs(hist - ref_hist)) <= 1e-3
    elif metric == "loglik":
        assert np.max(np.abs(hist - ref_hist) / np.abs(ref_hist)) <= 1e-6
    else:
        assert np.max(np.abs(hist - ref_hist)) <= 1e-6
    assert oracle.rel_l2(got, ref_u) <= 1e-4
    assert len(flux) == n
    total = float(c["d"].sum(dtype=np.float64))
    assert np.all(np.abs(flux - total) / total <= 1e-5)


def test_min_iter_and_never_stopping(torch):
    c = synth.make_config(0)
    say("stop min_iter / never")
    with rl.Plan(dev(torch, c["psf"])) as p:
        d = dev(torch, c["d"])
        u = dev(torch, c["u0"])
        p.iterate_until(d, u, 12, "change", 1e9, min_iter=5)  # would stop at once
        n, hist = p.stop()
        assert n == 5 and len(hist) == 5
        u = dev(torch, c["u0"])
        p.iterate_until(d, u, 12, "loglik", -1e300)
        n, hist = p.stop()
        assert n == 12 and len(hist) == 12
        v = dev(torch, c["u0"])
        p.iterate(d, v, 12)
        torch.cuda.synchronize()
        assert oracle.rel_l2(u.cpu().numpy(), v.cpu().numpy()) <= 1e-6
        u = dev(torch, c["u0"])
        p.iterate_until(d, u, 0, "change", 0.1)
        assert p.stop()[0] == 0
        with pytest.raises(rl.RLError):
            p.alpha()


def test_stop_zero_boundary(torch):
    shape, pshape = (20, 40, 36), (7, 9, 9)
    say("stop zero boundary")
    c = synth.small_case(shape, sigma_xyz=(1.2, 1.2, 2.0), seed=81)
    h = synth.gaussian_psf(pshape, (1.2, 1.2, 2.0))
    with rl.Plan(dev(torch, h), shape=shape, boundary="zero") as p:
        u = dev(torch, c["u0"])
        p.iterate_until(dev(torch, c["d"]), u, 40, "change", 9e-3)
        n, hist = p.stop()
        got = u.cpu().numpy()
    ref, _ = bo.rl_general(c["d"], h, c["u0"], n, boundary="zero")
    prev, _ = bo.rl_general(c["d"], h, c["u0"], n - 1, boundary="zero")
    # the oracle's changes fall from 1.07e-2 (iteration 5) to 7.9e-3 (iteration 6)
    assert n == 6 and hist[-1] < 9e-3 <= hist[-2]
    assert oracle.rel_l2(got, ref) <= 1e-4
    assert abs(hist[-1] - so.rel_change(ref, prev)) <= 1e-6


def test_stop_errors(torch):
    say("stop errors")
    c = synth.make_config(0)
    psf = dev(torch, c["psf"])
    d, u = dev(torch, c["d"]), dev(torch, c["u0"])
    with rl.Plan(psf) as p:
        with pytest.raises(rl.RLError) as ei:
            p.stop()
        assert ei.value.status == rl.RL_E_INVALID
        with pytest.raises(ValueError):
            p.iterate_until(d, u, 5, "psnr", 0.1)
        with pytest.raises(ValueError):
            p.iterate_until(d, u, 5, "ssim", 0.1)
        with pytest.raises(rl.RLError) as ei:
            rl.rl_iterate_stop(p.handle, d.data_ptr(), u.data_ptr(), 5, 9, 0.1)
        assert ei.value.status == rl.RL_E_INVALID
        with pytest.raises(rl.RLError) as ei:
            rl.rl_iterate_stop(p.handle, d.data_ptr(), u.data_ptr(), 5, rl.RL_STOP_CHANGE,
                               float("nan"))
        assert ei.value.status == rl.RL_E_INVALID
    with rl.Plan(psf, accel="biggs_andrews") as p:
        with pytest.raises(rl.RLError) as ei:
            p.iterate_until(d, u, 5, "change", 0.1)
        assert ei.value.status == rl.RL_E_UNSUPPORTED


def test_full_size_loglik_stop_as_benchmarked(torch):
    # the benchmark's stopping workload: the 128x256x256 volume, an autotuned plan,
    # the log-likelihood rule; the threshold sits halfway between two consecutive
    # improvements of the oracle's history so that the decision is unambiguous
    c = synth.make_config(1)
    say("full-size loglik stop", c["shape"])
    m = 7
    _, _, full = so.rl_stop(c["d"], c["psf"], c["u0"], m, "loglik", -1e300)
    tau = _threshold("loglik", full, 5)
    ref_u, ref_n, ref_hist = so.rl_stop(c["d"], c["psf"], c["u0"], m, "loglik", tau)
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        u = dev(torch, c["u0"])
        p.iterate_until(dev(torch, c["d"]), u, m, "loglik", tau)
        n, hist = p.stop()
        got = u.cpu().numpy()
    say("  oracle n", ref_n, "gpu n", n, "tau", tau)
    assert n == ref_n
    assert np.max(np.abs(hist - ref_hist) / np.abs(ref_hist)) <= 1e-6
    assert oracle.rel_l2(got, ref_u) <= 1e-5


@pytest.mark.parametrize("metric", ["change", "psnr", "ssim"])
def test_full_size_metric_histories_as_benchmarked(torch, metric):
    # the other benchmarked rules on the 128x256x256 volume (autotuned plan): with a
    # threshold that never fires, the metric after each of three iterations against
    # the oracle's (PSNR and SSIM against the ground truth, as the benchmark does)
    c = synth.make_config(1)
    truth = c["truth"].astype(np.float32)
    ref = truth if metric in ("psnr", "ssim") else None
    n = 3
    say("full-size history", metric)
    _, _, ref_hist = so.rl_stop(c["d"], c["psf"], c["u0"], n, metric, -1e300, reference=ref)
    with rl.Plan(dev(torch, c["psf"]), autotune=True) as p:
        u = dev(torch, c["u0"])
        p.iterate_until(dev(torch, c["d"]), u, n, metric, -1e300,
                        reference=dev(torch, truth) if ref is not None else None)
        k, hist = p.stop()
    say("  gpu", hist, "oracle", ref_hist)
    assert k == n and len(hist) == n
    tol = {"change": 1e-6, "psnr": 1e-3, "ssim": 1e-6}[metric]
    assert np.max(np.abs(hist - ref_hist)) <= tol
