"""Pins of the metric-guided stopping oracle.

* The scale-invariant PSNR against an independent route (numpy's least-squares
  polynomial fit of degree 1), its invariance under affine maps of the estimate,
  and its bound by the plain PSNR.
* The relative change on a closed form (a uniformly scaled estimate).
* Stopping never triggered reproduces the pinned plain oracle and its
  log-likelihood history; a triggered stop happens at the first iteration the
  full history says it should, with the estimate of the plain oracle after that
  many iterations.
* The delta PSF reaches its fixed point after one step, so the change criterion
  stops after the second.
* The FSC and SSIM histories are the FSC and SSIM oracles of each iterate.
* The last block plants plausible mistakes in the stopping oracle and checks
  that a pin catches each.
"""

import numpy as np
import pytest

import oracle
from oracle import stop_oracle as so


def rng(seed):
    return np.random.default_rng(seed)


def test_psnr_si_matches_polyfit_route():
    g = rng(1).uniform(0, 100, size=(6, 7, 8))
    u = 0.3 * g + 5.0 + rng(2).normal(0, 4.0, size=g.shape)
    a, b = np.polyfit(u.ravel(), g.ravel(), 1)
    mse = np.mean((a * u.ravel() + b - g.ravel()) ** 2)
    want = 20 * np.log10(g.max() - g.min()) - 10 * np.log10(mse)
    assert abs(so.psnr_si(u, g) - want) <= 1e-9


def test_psnr_si_affine_invariance_and_bound():
    g = rng(3).uniform(0, 50, size=(5, 6, 7))
    u = g + rng(4).normal(0, 2.0, size=g.shape)
    p = so.psnr_si(u, g)
    for a, b in ((2.0, 0.0), (0.5, 10.0), (-1.0, 3.0)):
        assert abs(so.psnr_si(a * u + b, g) - p) <= 1e-9
    plain = 20 * np.log10(g.max() - g.min()) - 10 * np.log10(np.mean((u - g) ** 2))
    assert p >= plain - 1e-12


def test_rel_change_closed_form():
    u = rng(5).uniform(1, 2, size=(4, 4, 4))
    for t in (0.5, -0.25, 1e-6):
        assert abs(so.rel_change((1 + t) * u, u) - abs(t)) <= 1e-12


def _case():
    shape = (8, 12, 10)
    h = rng(6).uniform(0, 1, size=shape) ** 3
    h[4, 6, 5] += 2.0
    truth = rng(7).uniform(5, 50, size=shape)
    d = rng(8).poisson(oracle.conv3d(truth, h)).astype(np.float64) + 1.0
    return d, h, np.full(shape, d.mean()), truth


def test_never_stopping_is_the_plain_oracle():
    d, h, u0, truth = _case()
    u, n, hist = so.rl_stop(d, h, u0, 9, "loglik", -np.inf)
    ur, _, ll = oracle.rl(d, h, u0, 9, with_loglik=True)
    assert n == 9 and np.allclose(u, ur, rtol=1e-13, atol=0)
    assert np.allclose(hist, ll, rtol=1e-13, atol=0)
    u, n, hist = so.rl_stop(d, h, u0, 7, "psnr", -np.inf, reference=truth)
    assert n == 7 and np.allclose(u, oracle.rl(d, h, u0, 7)[0], rtol=1e-13, atol=0)
    assert len(hist) == 7


@pytest.mark.parametrize("metric", ["loglik", "change", "psnr", "ssim"])
def test_stop_at_first_qualifying_iteration(metric, max_iter=30):
    d, h, u0, truth = _case()
    _, _, full = so.rl_stop(d, h, u0, max_iter, metric, -np.inf, reference=truth)
    if metric == "loglik":
        delta = np.diff(full) / np.abs(full[1:])          # index j -> check at iteration j + 1
        tau = float(np.median(delta))
        first = 1 + int(np.argmax(delta < tau))
        want_n = first
    elif metric == "change":
        tau = float(np.median(full))
        want_n = 1 + int(np.argmax(full < tau))
    else:                                                   # psnr, ssim
        delta = np.diff(full)                               # index j -> after iteration j + 2
        tau = float(np.median(delta))
        want_n = 2 + int(np.argmax(delta < tau))
    u, n, _ = so.rl_stop(d, h, u0, max_iter, metric, tau, reference=truth)
    assert n == want_n
    assert np.allclose(u, oracle.rl(d, h, u0, n)[0], rtol=1e-13, atol=0)
    # min_iter postpones the stop
    u, n2, _ = so.rl_stop(d, h, u0, max_iter, metric, tau, reference=truth, min_iter=want_n + 3)
    assert n2 >= want_n + 3


def test_loglik_improvements_are_non_negative():
    d, h, u0, _ = _case()
    # EM: the likelihood never decreases, so a threshold below every rounding step
    # never stops the iteration
    _, n, hist = so.rl_stop(d, h, u0, 15, "loglik", -1e-12)
    assert n == 15
    assert np.all(np.diff(hist) >= -1e-12 * np.abs(hist[1:]))


def test_fsc_metric_is_the_fsc_oracle_of_each_iterate():
    d, h, u0, _ = _case()
    u, n, hist = so.rl_stop(d, h, u0, 4, "fsc", -1e300, nbins=8)
    assert n == 4 and len(hist) == 4
    for k in range(4):
        uk = oracle.rl(d, h, u0, k + 1)[0]
        a, b = uk[0::2, 0::2, 0::2], uk[1::2, 1::2, 1::2]
        assert hist[k] == oracle.resolution(oracle.fsc(a, b, 8), 8)


def test_delta_psf_change_stops_after_fixed_point():
    shape = (4, 6, 6)
    d = rng(9).uniform(1, 10, size=shape)
    h = np.zeros(shape)
    h[2, 3, 3] = 1.0
    u, n, hist = so.rl_stop(d, h, np.full(shape, 2.0), 10, "change", 1e-9)
    assert n == 2 and hist[1] < 1e-9 and hist[0] > 0.1
    assert np.allclose(u, d, rtol=1e-12)


def test_ssim_metric_is_the_ssim_oracle_of_each_iterate():
    d, h, u0, truth = _case()
    u, n, hist = so.rl_stop(d, h, u0, 4, "ssim", -1e300, reference=truth)
    assert n == 4 and len(hist) == 4
    for k in range(4):
        uk = oracle.rl(d, h, u0, k + 1)[0]
        assert hist[k] == oracle.ssim(uk, truth)


# ---------------------------------------------------------------------------
# Planted mistakes: each must make one of the pins above fail.
# ---------------------------------------------------------------------------
from mutation import mutate  # noqa: E402


def _pins_hold():
    """Re-run a compact set of the pins; False if any fails."""
    tests = [test_psnr_si_matches_polyfit_route, test_psnr_si_affine_invariance_and_bound,
             test_rel_change_closed_form, test_never_stopping_is_the_plain_oracle,
             test_fsc_metric_is_the_fsc_oracle_of_each_iterate,
             test_ssim_metric_is_the_ssim_oracle_of_each_iterate,
             test_delta_psf_change_stops_after_fixed_point]
    tests += [lambda m=m: test_stop_at_first_qualifying_iteration(m, max_iter=16)
              for m in ("loglik", "change", "psnr", "ssim")]
    try:
        for t in tests:
            t()
    except Exception:
        return False
    return True


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("func,old,new", [
    # change relative to the new estimate
    ("rel_change", "np.linalg.norm(b.ravel())", "np.linalg.norm(a.ravel())"),
    # PSNR without the affine fit
    ("psnr_si", "sse = cgg - (cug * cug / cuu if cuu > 0 else 0.0)",
     "sse = float(np.sum((u - g) ** 2))"),
    # dynamic range of the estimate instead of the reference
    ("psnr_si", "rng = float(g.max() - g.min())", "rng = float(u.max() - u.min())"),
    # absolute instead of relative log-likelihood improvement
    ("rl_stop", "(hist[k] - hist[k - 1]) / abs(hist[k]) < threshold",
     "(hist[k] - hist[k - 1]) < threshold"),
    # log-likelihood checked before there is a previous value
    ("rl_stop", "if k >= 1 and k >= min_iter:", "if k >= min_iter:"),
    # the PSNR value itself compared with the threshold, not its improvement
    ("rl_stop", "hist.append(psnr_si(u_new, reference))\n            stop = k >= 1 and hist[k] - hist[k - 1] < threshold",
     "hist.append(psnr_si(u_new, reference))\n            stop = k >= 1 and hist[k] < threshold"),
    # SSIM with its arguments swapped (range taken from the estimate)
    ("rl_stop", "ssim_oracle.ssim(u_new, reference)", "ssim_oracle.ssim(reference, u_new)"),
    # the stop returns the estimate from before the last iteration
    ("rl_stop", "u = u_new\n        if stop and n_done >= min_iter:\n            break",
     "if stop and n_done >= min_iter:\n            break\n        u = u_new"),
    # min_iter ignored by the change, PSNR, SSIM and FSC rules
    ("rl_stop", "if stop and n_done >= min_iter:", "if stop:"),
    # the change measured against the starting estimate
    ("rl_stop", "hist.append(rel_change(u_new, u))", "hist.append(rel_change(u_new, u0))"),
])
def test_planted_mistake_is_caught(monkeypatch, func, old, new):
    monkeypatch.setattr(so, func, mutate(so, func, old, new))
    assert not _pins_hold(), (func, new)
