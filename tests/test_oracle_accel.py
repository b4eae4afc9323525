"""Pins of the Biggs-Andrews oracle to results that do not come from it.

* Closed form: on the linear contraction psi(y) = a + rho (y - a), applied
  elementwise, the extrapolation with unclipped alphas gives
  alpha_k = rho^(k-1) for k >= 2 and x_n = a + rho^(n(n-1)/2 + 1) (x_0 - a) for
  n >= 1 (the exponents of the predictions are the triangular numbers).
* Reduction: for n_iter <= 2 no alpha is non-zero, so the accelerated
  Richardson-Lucy equals the plain one (itself pinned in test_oracle_pins).
* Richardson-Lucy invariants that hold from any non-negative starting point:
  flux conservation, non-negativity, the delta-PSF fixed point.
* The prediction is clamped at zero whenever the raw extrapolation goes negative.
The last block plants plausible mistakes in the extrapolation and checks that a
pin catches each.
"""

import numpy as np
import pytest

import oracle
from oracle import accel_oracle


def rng_psf(shape, seed):
    h = np.random.default_rng(seed).uniform(0.0, 1.0, size=shape)
    h.flat[0] += 0.5
    return h


def _delta(shape):
    h = np.zeros(shape)
    h[tuple(n // 2 for n in shape)] = 1.0
    return h


def _contraction_case(extrap, n):
    rng = np.random.default_rng(40)
    a = rng.uniform(4.0, 6.0, size=(3, 5))
    e0 = rng.uniform(-1.0, 1.0, size=(3, 5))
    rho = 0.8
    psi = lambda y: a + rho * (y - a)  # noqa: E731
    x, alphas = extrap(psi, a + e0, n)
    want_x = a + rho ** (n * (n - 1) // 2 + 1) * e0
    want_alpha = np.array([0.0 if k < 2 else rho ** (k - 1) for k in range(n)])
    return x, alphas, want_x, want_alpha


@pytest.mark.parametrize("n", [1, 2, 3, 4, 5, 6])
def test_closed_form_on_linear_contraction(n):
    x, alphas, want_x, want_alpha = _contraction_case(accel_oracle.extrapolate, n)
    assert np.allclose(x, want_x, rtol=0, atol=1e-12)
    assert np.allclose(alphas, want_alpha, rtol=0, atol=1e-12)


@pytest.mark.parametrize("n", [0, 1, 2])
def test_first_two_iterations_are_plain_rl(n):
    shape = (4, 6, 8)
    h = rng_psf(shape, 41)
    d = np.random.default_rng(42).uniform(1, 10, size=shape)
    u0 = np.full(shape, d.mean())
    ua, fa, al = accel_oracle.rl_accel(d, h, u0, n)
    up, fp, _ = oracle.rl(d, h, u0, n)
    assert np.array_equal(ua, up) and np.array_equal(fa, fp)
    assert np.all(al == 0.0)


def test_flux_nonneg_and_alpha_range():
    shape = (6, 8, 10)
    h = rng_psf(shape, 43)
    d = np.random.default_rng(44).uniform(1, 50, size=shape)
    u0 = np.full(shape, d.mean())
    u, flux, alphas = accel_oracle.rl_accel(d, h, u0, 12)
    assert np.all(u >= 0)
    assert np.allclose(flux, d.sum(), rtol=1e-12, atol=0)
    assert np.all((alphas >= 0) & (alphas <= 1))
    assert np.any(alphas[2:] > 0)  # the acceleration is active


def test_delta_psf_fixed_point():
    shape = (4, 4, 6)
    d = np.random.default_rng(45).uniform(1, 10, size=shape)
    u, flux, alphas = accel_oracle.rl_accel(d, _delta(shape), np.full(shape, 3.0), 6)
    assert np.allclose(u, d, rtol=1e-13, atol=0)
    # after the first step nothing changes any more, so g = 0 and alpha falls back to 0
    assert np.all(alphas[3:] == 0.0)


def test_prediction_clamped_at_zero():
    # one coordinate settles fast towards 0 while a slow one sets alpha near 1: the raw
    # prediction of the fast one overshoots below zero and the clamped one is 0
    target = np.array([0.0, 4.0])
    rho = np.array([0.1, 0.95])
    psi = lambda y: target + rho * (y - target)  # noqa: E731
    trace = []
    accel_oracle.extrapolate(psi, np.array([3.0, 0.0]), 8, trace=trace)
    raws = np.array([r for r, _ in trace])
    ys = np.array([y for _, y in trace])
    assert np.all(ys >= 0)
    assert np.any(raws < 0)
    assert np.array_equal(ys, np.maximum(raws, 0))


def test_accelerated_likelihood_ahead_of_plain():
    # the point of the method: at equal iteration counts the extrapolated run has gone
    # further up the Poisson likelihood than the plain one (checked on a blurred scene)
    shape = (8, 16, 16)
    rng = np.random.default_rng(46)
    x = np.full(shape, 5.0)
    x[2:5, 4:9, 6:12] += 200.0
    x[6, 12, 3] += 800.0
    zz, yy, xx = np.meshgrid(*[np.arange(n) - n // 2 for n in shape], indexing="ij")
    h = np.exp(-0.5 * ((zz / 2.0) ** 2 + (yy / 1.5) ** 2 + (xx / 1.5) ** 2))
    d = rng.poisson(oracle.conv3d(x, h)).astype(np.float64)
    u0 = np.full(shape, d.mean())
    K = oracle.otf(h)
    n = 15
    ua, _, _ = accel_oracle.rl_accel(d, h, u0, n)
    up, _, _ = oracle.rl(d, h, u0, n)
    assert oracle.loglik(d, oracle.forward(ua, K)) > oracle.loglik(d, oracle.forward(up, K))


# --------------------------------------------------------------------------
# Planted mistakes in the extrapolation
# --------------------------------------------------------------------------

def _make_mutant(kind):
    def extrap(psi, x0, n_iter, clamp=True, trace=None):
        x = np.array(x0, dtype=np.float64)
        x_prev = None
        g1 = g2 = None
        alphas = []
        for k in range(n_iter):
            alpha = 0.0
            if g2 is not None and np.sum(g2 * g2) > 0:
                if kind == "alpha uses g_k-1 twice":
                    num = np.sum(g1 * g1)
                else:
                    num = np.sum(g1 * g2)
                den = np.sum(g1 * g1) if kind == "alpha normalised by g_k-1" else np.sum(g2 * g2)
                alpha = min(max(num / den, 0.0), 1.0)
            if kind == "alpha starts one iteration early" and g1 is not None and g2 is None:
                alpha = 0.5
            alphas.append(alpha)
            if x_prev is None:
                h = np.zeros_like(x)
            elif kind == "step sign reversed":
                h = x_prev - x
            else:
                h = x - x_prev
            y = np.maximum(x + alpha * h, 0.0)
            x_next = psi(y)
            g = x_next - (x if kind == "change measured from x_k" else y)
            g2, g1 = g1, g
            x_prev, x = x, x_next
        return x, np.array(alphas)
    return extrap


@pytest.mark.parametrize("kind", ["alpha uses g_k-1 twice", "alpha normalised by g_k-1",
                                  "alpha starts one iteration early", "step sign reversed",
                                  "change measured from x_k"])
def test_planted_mistake_is_caught(kind):
    caught = False
    for n in range(1, 7):
        x, alphas, want_x, want_alpha = _contraction_case(_make_mutant(kind), n)
        if not (np.allclose(x, want_x, rtol=0, atol=1e-12)
                and np.allclose(alphas, want_alpha, rtol=0, atol=1e-12)):
            caught = True
    assert caught, kind


def test_unmutated_copy_passes():
    for n in range(1, 7):
        x, alphas, want_x, want_alpha = _contraction_case(_make_mutant("none"), n)
        assert np.allclose(x, want_x, rtol=0, atol=1e-12)
        assert np.allclose(alphas, want_alpha, rtol=0, atol=1e-12)
