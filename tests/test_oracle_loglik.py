"""Pins of the oracle's Poisson log-likelihood (paper §4.3, paragraph
"Richardson-Lucy algorithm": the iteration maximises the likelihood under
Poisson noise) to values that do not come from the oracle itself: a hand-worked
example with its guarded case (tests/golden/loglik_worked_1x1x4.txt), the closed
form of constant data, and scipy's Poisson log-probability.  The last block
plants plausible mistakes in ``loglik`` and checks that a pin catches each."""

import math
import os
from fractions import Fraction

import numpy as np
import pytest
from scipy import special, stats

import oracle
from oracle import rl_oracle

from mutation import mutate

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "loglik_worked_1x1x4.txt")


def _golden():
    vals = {}
    with open(GOLDEN) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = [float(Fraction(t)) for t in rest]
    return vals


def _worked_case():
    h = np.array([0.0, 0.0, 3.0, 1.0]).reshape(1, 1, 4)
    d = np.array([1.0, 2.0, 3.0, 6.0]).reshape(1, 1, 4)
    return h, d, np.full((1, 1, 4), 3.0)


def _pins_hold():
    """The pins below as one predicate (for the planted-mistake tests)."""
    try:
        g = _golden()
        h, d, u0 = _worked_case()
        _, _, ll = rl_oracle.rl(d, h, u0, 2, with_loglik=True)
        if not np.allclose(ll, [g["l0"][0], g["l1"][0]], rtol=1e-13, atol=0):
            return False
        gd = np.array(g["guard_d"]).reshape(1, 1, 4)
        gq = np.array(g["guard_q"]).reshape(1, 1, 4)
        if not math.isclose(rl_oracle.loglik(gd, gq), g["guard_l"][0], rel_tol=1e-13):
            return False
        c = 6.5
        shape = (3, 4, 5)
        dc = np.full(shape, c)
        _, _, llc = rl_oracle.rl(dc, np.random.default_rng(1).uniform(size=shape), dc, 1,
                                 with_loglik=True)
        if not math.isclose(llc[0], dc.size * (c * math.log(c) - c), rel_tol=1e-12):
            return False
        return _scipy_pin(rl_oracle.loglik)
    except Exception:
        return False


def _scipy_pin(fn):
    """loglik == sum over q > eps of (poisson.logpmf(d; q) + log d!) on integer data."""
    rng = np.random.default_rng(7)
    shape = (4, 5, 6)
    q = rng.uniform(0.5, 40.0, size=shape)
    q.flat[::7] = 0.0            # guarded voxels (q <= eps)
    q.flat[3] = -2.0             # round-off can leave q slightly negative: guarded too
    d = rng.poisson(12.0, size=shape).astype(np.float64)
    d.flat[::5] = 0.0            # zero counts: their term is -q
    ok = q > oracle.EPS
    ref = float(np.sum(stats.poisson.logpmf(d[ok], q[ok]) + special.gammaln(d[ok] + 1.0)))
    return math.isclose(fn(d, q), ref, rel_tol=1e-12)


def test_worked_example_values():
    g = _golden()
    h, d, u0 = _worked_case()
    _, _, ll = oracle.rl(d, h, u0, 2, with_loglik=True)
    assert ll[0] == pytest.approx(g["l0"][0], rel=1e-13)
    assert ll[1] == pytest.approx(g["l1"][0], rel=1e-13)
    # the q the hand derivation used is the oracle's blur of u0 and u1
    K = oracle.otf(h)
    u1, _, _ = oracle.rl(d, h, u0, 1)
    assert np.allclose(oracle.forward(u0, K).ravel(), g["q0"], rtol=1e-14)
    assert np.allclose(oracle.forward(u1, K).ravel(), g["q1"], rtol=1e-14)


def test_guarded_voxels_and_zero_counts():
    g = _golden()
    d = np.array(g["guard_d"]).reshape(1, 1, 4)
    q = np.array(g["guard_q"]).reshape(1, 1, 4)
    assert oracle.loglik(d, q) == pytest.approx(g["guard_l"][0], rel=1e-13)


@pytest.mark.parametrize("c", [0.25, 1.0, 6.5, 1000.0])
def test_constant_data_closed_form(c):
    # d = u = c with any unit-sum PSF: q = c everywhere, so l = N (c log c - c)
    shape = (3, 4, 5)
    h = np.random.default_rng(2).uniform(size=shape)
    dc = np.full(shape, c)
    _, _, ll = oracle.rl(dc, h, dc, 3, with_loglik=True)
    assert np.allclose(ll, dc.size * (c * math.log(c) - c), rtol=1e-12, atol=0)


def test_matches_scipy_poisson_logpmf():
    assert _scipy_pin(oracle.loglik)


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("name,old,new", [
    ("the -sum q term dropped", " - np.sum(qq)", ""),
    ("q summed over every voxel, not only q > eps", "np.sum(qq)", "np.sum(q)"),
    ("log d in place of log q", "np.log(qq[pos])", "np.log(dd[pos])"),
    ("guard taken as q >= 0", "ok = q > eps", "ok = q >= 0"),
    ("zero counts left out of the -q sum", "np.sum(qq))", "np.sum(qq[pos]))"),
])
def test_planted_mistake_is_caught(monkeypatch, name, old, new):
    monkeypatch.setattr(rl_oracle, "loglik", mutate(rl_oracle, "loglik", old, new))
    assert not _pins_hold(), name
