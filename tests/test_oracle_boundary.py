"""Pins of the small-PSF and zero-boundary oracle to results that do not come from it.

* An independent library: scipy.signal's full linear convolution, cropped at the
  PSF centre, equals the zero-boundary convolution; the correlation equals the
  full convolution with the flipped PSF, cropped accordingly.
* Brute-force sums written from the definition (pure Python) on tiny volumes.
* A PSF smaller than the volume, periodic boundary, equals the pinned
  same-shape oracle applied to that PSF zero-padded with its centre moved to
  floor(n/2).
* Adjointness, independence of the padded grid size, the delta-PSF fixed point,
  non-negativity and flux conservation of the zero-boundary iteration.
The last block plants mistakes and checks that a pin catches each.
"""

import itertools

import numpy as np
import pytest
from scipy import signal

import oracle
from oracle import boundary_oracle as bo


def rng(seed):
    return np.random.default_rng(seed)


def rand_psf(shape, seed):
    h = rng(seed).uniform(0, 1, size=shape)
    h.flat[-1] += 0.7  # asymmetric
    return h


def close(a, b, tol=1e-12):
    a, b = np.asarray(a), np.asarray(b)
    return np.max(np.abs(a - b)) <= tol * max(1.0, np.max(np.abs(b)))


SHAPES = [((6, 7, 8), (3, 4, 5)), ((5, 8, 6), (5, 8, 6)), ((4, 6, 9), (1, 2, 3)),
          ((8, 4, 4), (4, 1, 3)), ((1, 9, 10), (1, 5, 4))]


def _scipy_conv_zero(x, h):
    hn = h / h.sum()
    full = signal.convolve(x, hn, mode="full", method="direct")
    c = [p // 2 for p in h.shape]
    return full[tuple(slice(ci, ci + n) for ci, n in zip(c, x.shape))]


def _scipy_corr_zero(y, h):
    hn = h / h.sum()
    full = signal.convolve(y, hn[::-1, ::-1, ::-1], mode="full", method="direct")
    c = [p // 2 for p in h.shape]
    off = [p - 1 - ci for p, ci in zip(h.shape, c)]
    return full[tuple(slice(o, o + n) for o, n in zip(off, y.shape))]


@pytest.mark.parametrize("shape,pshape", SHAPES)
def test_zero_boundary_matches_scipy_full_convolution(shape, pshape):
    x = rng(1).uniform(0, 5, size=shape)
    h = rand_psf(pshape, 2)
    assert close(bo.conv_zero(x, h), _scipy_conv_zero(x, h))
    assert close(bo.corr_zero(x, h), _scipy_corr_zero(x, h))
    assert close(bo.conv_zero_direct(x, h), _scipy_conv_zero(x, h))
    assert close(bo.corr_zero_direct(x, h), _scipy_corr_zero(x, h))


def _brute(x, h, periodic, adjoint):
    hn = h / h.sum()
    c = [p // 2 for p in h.shape]
    out = np.zeros(x.shape)
    for i in itertools.product(*[range(n) for n in x.shape]):
        s = 0.0
        for m in itertools.product(*[range(p) for p in h.shape]):
            k = [mi - ci for mi, ci in zip(m, c)]
            j = [ii + ki if adjoint else ii - ki for ii, ki in zip(i, k)]
            if periodic:
                j = [jj % n for jj, n in zip(j, x.shape)]
            elif any(jj < 0 or jj >= n for jj, n in zip(j, x.shape)):
                continue
            s += hn[m] * x[tuple(j)]
        out[i] = s
    return out


@pytest.mark.parametrize("shape,pshape", [((3, 4, 5), (2, 3, 3)), ((4, 3, 4), (4, 3, 4)),
                                          ((2, 5, 4), (1, 2, 4))])
def test_brute_force_sums(shape, pshape):
    x = rng(3).uniform(0, 5, size=shape)
    h = rand_psf(pshape, 4)
    assert close(bo.conv_zero(x, h), _brute(x, h, False, False))
    assert close(bo.corr_zero(x, h), _brute(x, h, False, True))
    assert close(bo.conv_periodic(x, h), _brute(x, h, True, False))
    assert close(bo.corr_periodic(x, h), _brute(x, h, True, True))


@pytest.mark.parametrize("shape,pshape", SHAPES)
def test_small_psf_periodic_equals_padded_same_shape_psf(shape, pshape):
    x = rng(5).uniform(0, 5, size=shape)
    h = rand_psf(pshape, 6)
    big = np.zeros(shape)
    start = [n // 2 - p // 2 for n, p in zip(shape, pshape)]
    big[tuple(slice(s, s + p) for s, p in zip(start, pshape))] = h
    assert close(bo.conv_periodic(x, h), oracle.conv3d(x, big))
    assert close(bo.corr_periodic(x, h), oracle.adjoint(x, oracle.otf(big)))


@pytest.mark.parametrize("shape,pshape", SHAPES)
def test_pointwise_zero_conv(shape, pshape):
    x = rng(15).uniform(0, 5, size=shape)
    h = rand_psf(pshape, 16)
    full = _scipy_conv_zero(x, h)
    pts = [tuple(int(v) for v in rng(17 + k).integers(0, shape)) for k in range(6)]
    pts += [(0, 0, 0), tuple(n - 1 for n in shape)]
    assert close(bo.conv_zero_at(x, h, pts), np.array([full[p] for p in pts]))


@pytest.mark.parametrize("shape,pshape", SHAPES)
def test_adjoint_and_pad_independence(shape, pshape):
    x = rng(7).uniform(0, 5, size=shape)
    y = rng(8).uniform(0, 5, size=shape)
    h = rand_psf(pshape, 9)
    assert abs(np.vdot(bo.conv_zero(x, h), y) - np.vdot(x, bo.corr_zero(y, h))) <= 1e-10 * abs(
        np.vdot(x, y))
    assert close(bo.conv_zero(x, h), bo.conv_zero(x, h, extra_pad=7))
    assert close(bo.corr_zero(y, h), bo.corr_zero(y, h, extra_pad=3))


def test_zero_boundary_rl_invariants():
    shape = (6, 8, 10)
    h = rand_psf((3, 5, 5), 10)
    d = rng(11).uniform(1, 40, size=shape)
    u0 = np.full(shape, d.mean())
    u, flux = bo.rl_general(d, h, u0, 8, boundary="zero")
    assert np.all(u >= 0)
    assert np.allclose(flux, d.sum(), rtol=1e-12, atol=0)
    # delta PSF: H = I on either boundary, the data are a fixed point
    delta = np.zeros((3, 3, 3))
    delta[1, 1, 1] = 2.0
    u, _ = bo.rl_general(d, delta, u0, 3, boundary="zero")
    assert close(u, d, 1e-13)
    # the same-shape periodic case is the pinned plain oracle
    hp = rand_psf(shape, 12)
    up, _ = bo.rl_general(d, hp, u0, 4, boundary="periodic")
    ur, _, _ = oracle.rl(d, hp, u0, 4)
    assert close(up, ur, 1e-11)


def test_zero_boundary_differs_from_periodic_only_near_the_border():
    shape = (12, 12, 12)
    h = rand_psf((3, 3, 3), 13)
    x = rng(14).uniform(0, 5, size=shape)
    a, b = bo.conv_zero(x, h), bo.conv_periodic(x, h)
    inner = (slice(1, -1),) * 3
    assert close(a[inner], b[inner])
    assert not close(a, b)


# --------------------------------------------------------------------------
# Planted mistakes
# --------------------------------------------------------------------------

def _pins_hold():
    try:
        for shape, pshape in SHAPES[:3]:
            x = rng(20).uniform(0, 5, size=shape)
            h = rand_psf(pshape, 21)
            if not close(bo.conv_zero(x, h), _scipy_conv_zero(x, h)):
                return False
            if not close(bo.corr_zero(x, h), _scipy_corr_zero(x, h)):
                return False
            big = np.zeros(shape)
            start = [n // 2 - p // 2 for n, p in zip(shape, pshape)]
            big[tuple(slice(s, s + p) for s, p in zip(start, pshape))] = h
            if not close(bo.conv_periodic(x, h), oracle.conv3d(x, big)):
                return False
        return True
    except Exception:
        return False


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


def _mut_centre_ceil(shape):
    return tuple((int(n) + 1) // 2 for n in shape)


def _mut_grid_too_small(shape, psf_shape, extra=0):
    return tuple(int(n) + extra for n in shape)  # wrapped terms reach the volume


def _mut_embed_unnormalised(h):
    return np.asarray(h, dtype=np.float64)


@pytest.mark.parametrize("attr,mut", [("psf_centre", _mut_centre_ceil),
                                      ("_padded_grid", _mut_grid_too_small),
                                      ("_normalised", _mut_embed_unnormalised)])
def test_planted_mistake_is_caught(monkeypatch, attr, mut):
    monkeypatch.setattr(bo, attr, mut)
    assert not _pins_hold(), attr
