"""Pins of the FP64 oracle to mathematics that does not come from the oracle itself.

The paper prints no worked Richardson-Lucy numbers (§4.3 describes the method in
one paragraph), so every pin here is a closed form, an invariant, an independent
library, a brute-force sum written from the definition, or exact rational
arithmetic.  The last block plants plausible mistakes in the oracle and checks
that at least one pin catches each of them.
"""

import itertools
import os
from fractions import Fraction

import numpy as np
import pytest

import oracle
from oracle import rl_oracle

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def rng_psf(shape, seed, zero_frac=0.0):
    rng = np.random.default_rng(seed)
    h = rng.uniform(0.0, 1.0, size=shape)
    if zero_frac:
        h[rng.uniform(size=shape) < zero_frac] = 0.0
    h.flat[0] += 0.5  # asymmetric, strictly positive sum
    return h


def rng_data(shape, seed, lo=1.0, hi=10.0):
    return np.random.default_rng(seed).uniform(lo, hi, size=shape)


# --------------------------------------------------------------------------
# Independent re-derivations used as pins (pure Python, from the definitions)
# --------------------------------------------------------------------------

def brute_conv(x, h):
    """(Hx)[m] = sum_j h[j]/S * x[(m - (j - c)) mod n], written as loops over the raw PSF."""
    nz, ny, nx = x.shape
    cz, cy, cx = nz // 2, ny // 2, nx // 2
    s = float(np.sum(h))
    out = np.zeros(x.shape)
    for m in itertools.product(range(nz), range(ny), range(nx)):
        acc = 0.0
        for j in itertools.product(range(nz), range(ny), range(nx)):
            w = h[j]
            if w == 0:
                continue
            src = ((m[0] - (j[0] - cz)) % nz, (m[1] - (j[1] - cy)) % ny, (m[2] - (j[2] - cx)) % nx)
            acc += w * x[src]
        out[m] = acc / s
    return out


def brute_corr(y, h):
    """(H^T y)[m] = sum_j h[j]/S * y[(m + (j - c)) mod n]."""
    nz, ny, nx = y.shape
    cz, cy, cx = nz // 2, ny // 2, nx // 2
    s = float(np.sum(h))
    out = np.zeros(y.shape)
    for m in itertools.product(range(nz), range(ny), range(nx)):
        acc = 0.0
        for j in itertools.product(range(nz), range(ny), range(nx)):
            w = h[j]
            if w == 0:
                continue
            src = ((m[0] + (j[0] - cz)) % nz, (m[1] + (j[1] - cy)) % ny, (m[2] + (j[2] - cx)) % nx)
            acc += w * y[src]
        out[m] = acc / s
    return out


def exact_rl(d, h, u0, n_iter):
    """Richardson-Lucy in exact rational arithmetic (Fractions), by definition."""
    shape = d.shape
    nz, ny, nx = shape
    cz, cy, cx = nz // 2, ny // 2, nx // 2
    idx = list(itertools.product(range(nz), range(ny), range(nx)))
    hs = {j: Fraction(int(h[j])) for j in idx if h[j] != 0}
    S = sum(hs.values())
    dd = {m: Fraction(int(d[m])) for m in idx}
    u = {m: Fraction(u0[m]) for m in idx}
    for _ in range(n_iter):
        q = {}
        for m in idx:
            q[m] = sum(w * u[((m[0] - (j[0] - cz)) % nz, (m[1] - (j[1] - cy)) % ny,
                                (m[2] - (j[2] - cx)) % nx)] for j, w in hs.items()) / S
        r = {m: (dd[m] / q[m] if q[m] > 0 else Fraction(0)) for m in idx}
        newu = {}
        for m in idx:
            c = sum(w * r[((m[0] + (j[0] - cz)) % nz, (m[1] + (j[1] - cy)) % ny,
                             (m[2] + (j[2] - cx)) % nx)] for j, w in hs.items()) / S
            newu[m] = u[m] * max(c, Fraction(0))
        u = newu
    out = np.zeros(shape)
    for m in idx:
        out[m] = float(u[m])
    return out


def close(a, b, tol):
    return oracle.rel_l2(a, b) <= tol


# --------------------------------------------------------------------------
# DFT
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 8, 6), (8, 8, 4), (1, 1, 7), (32, 64, 64)])
def test_dft_matches_numpy_fft(shape):
    x = np.random.default_rng(1).standard_normal(shape) + 1j * np.random.default_rng(2).standard_normal(shape)
    X = oracle.dft3(x)
    ref = np.fft.fftn(x)
    assert np.max(np.abs(X - ref)) <= 1e-12 * np.max(np.abs(ref)) * np.sqrt(x.size)
    back = oracle.idft3(X)
    assert np.max(np.abs(back - x)) <= 1e-12 * np.max(np.abs(x)) * np.sqrt(x.size)


def test_dft_closed_forms():
    # delta -> all ones; constant -> N * delta; single frequency -> delta at that frequency
    shape = (3, 4, 6)
    d = np.zeros(shape); d[0, 0, 0] = 1
    assert np.allclose(oracle.dft3(d), np.ones(shape), atol=1e-14)
    one = np.ones(shape)
    ref = np.zeros(shape, complex); ref[0, 0, 0] = one.size
    assert np.allclose(oracle.dft3(one), ref, atol=1e-12)
    kz, ky, kx = 1, 3, 2
    z, y, x = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    wave = np.exp(2j * np.pi * (kz * z / 3 + ky * y / 4 + kx * x / 6))
    ref = np.zeros(shape, complex); ref[kz, ky, kx] = one.size
    assert np.allclose(oracle.dft3(wave), ref, atol=1e-11)


# --------------------------------------------------------------------------
# Convolution and adjoint
# --------------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(4, 6, 5), (3, 8, 6), (8, 8, 4), (2, 3, 4), (1, 5, 6)])
def test_conv_theorem_vs_brute_force(shape):
    h = rng_psf(shape, 3, zero_frac=0.3)
    x = rng_data(shape, 4)
    ref = brute_conv(x, h)
    assert close(oracle.conv3d(x, h), ref, 1e-12)
    assert close(oracle.conv_direct(x, h), ref, 1e-12)
    K = oracle.otf(h)
    assert close(oracle.adjoint(x, K), brute_corr(x, h), 1e-12)
    assert close(oracle.corr_direct(x, h), brute_corr(x, h), 1e-12)


def test_conv_direct_at_matches_brute():
    shape = (4, 6, 8)
    h = rng_psf(shape, 5)
    x = rng_data(shape, 6)
    ref = brute_conv(x, h)
    pts = [(0, 0, 0), (3, 5, 7), (1, 2, 3), (2, 0, 7)]
    got = oracle.conv_direct_at(x, h, pts)
    assert np.allclose(got, [ref[p] for p in pts], rtol=1e-13, atol=0)


def test_adjointness():
    shape = (6, 5, 8)
    h = rng_psf(shape, 7)
    K = oracle.otf(h)
    x, y = rng_data(shape, 8), rng_data(shape, 9)
    lhs = float(np.sum(oracle.forward(x, K) * y))
    rhs = float(np.sum(x * oracle.adjoint(y, K)))
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_psf_validation():
    shape = (2, 2, 2)
    with pytest.raises(ValueError):
        oracle.check_psf(np.zeros(shape))
    bad = np.ones(shape); bad[0, 0, 0] = -1
    with pytest.raises(ValueError):
        oracle.check_psf(bad)
    bad = np.ones(shape); bad[1, 1, 1] = np.nan
    with pytest.raises(ValueError):
        oracle.check_psf(bad)


# --------------------------------------------------------------------------
# Richardson-Lucy
# --------------------------------------------------------------------------

def test_golden_hand_worked_example():
    vals = {}
    with open(os.path.join(GOLDEN, "rl_worked_1x1x4.txt")) as f:
        for line in f:
            line = line.strip()
            if not line or line.startswith("#"):
                continue
            key, *rest = line.split()
            vals[key] = [Fraction(t) for t in rest]
    shape = tuple(int(v) for v in vals["shape"])
    h = np.array([float(v) for v in vals["psf"]]).reshape(shape)
    d = np.array([float(v) for v in vals["d"]]).reshape(shape)
    u0 = np.array([float(v) for v in vals["u0"]]).reshape(shape)
    for n, key in ((1, "u1"), (2, "u2")):
        u, flux, _ = oracle.rl(d, h, u0, n)
        ref = np.array([float(v) for v in vals[key]]).reshape(shape)
        assert np.allclose(u, ref, rtol=1e-14, atol=1e-14), (key, u, ref)
        assert abs(flux[-1] - 12.0) <= 1e-13


@pytest.mark.parametrize("shape,n_iter", [((2, 3, 4), 2), ((3, 2, 5), 2), ((1, 4, 6), 3)])
def test_rl_exact_rational_brute_force(shape, n_iter):
    rng = np.random.default_rng(11)
    h = rng.integers(0, 6, size=shape).astype(float)
    h.flat[-1] += 1  # never all zero; asymmetric in general
    d = rng.integers(1, 20, size=shape).astype(float)
    u0 = np.full(shape, Fraction(int(d.sum()), d.size), dtype=object)
    ref = exact_rl(d, h, u0, n_iter)
    u, _, _ = oracle.rl(d, h, u0.astype(float), n_iter)
    assert close(u, ref, 1e-13)


def test_rl_dft_route_equals_direct_route():
    shape = (6, 8, 10)
    h = rng_psf(shape, 12, zero_frac=0.5)
    d = rng_data(shape, 13)
    u0 = np.full(shape, d.mean())
    u, _, _ = oracle.rl(d, h, u0, 5)
    ud = oracle.rl_direct(d, h, u0, 5)
    assert close(u, ud, 1e-12)


def _delta(shape, offset=(0, 0, 0)):
    h = np.zeros(shape)
    c = oracle.psf_centre(shape)
    h[tuple((c[i] + offset[i]) % shape[i] for i in range(3))] = 1.0
    return h


def test_delta_psf_fixed_point():
    shape = (4, 6, 8)
    d = rng_data(shape, 14)
    u0 = np.full(shape, d.mean())
    K = oracle.otf(_delta(shape))
    x = rng_data(shape, 15)
    assert np.allclose(oracle.forward(x, K), x, rtol=1e-14, atol=1e-13)
    for n in (1, 2, 5):
        u, _, _ = oracle.rl(d, _delta(shape), u0, n)
        assert np.allclose(u, d, rtol=1e-13, atol=0)


@pytest.mark.parametrize("s", [(1, 0, 0), (0, 1, 2), (1, -1, 3), (2, 2, -1)])
def test_shifted_delta_inverts_in_one_step(s):
    shape = (4, 6, 8)
    d = rng_data(shape, 16)
    u0 = np.full(shape, d.mean())
    h = _delta(shape, s)
    K = oracle.otf(h)
    x = rng_data(shape, 17)
    # H is the shift by s: (Hx)[m] = x[m - s]
    assert np.allclose(oracle.forward(x, K), np.roll(x, s, axis=(0, 1, 2)), rtol=1e-13, atol=1e-12)
    u1, _, _ = oracle.rl(d, h, u0, 1)
    # one step gives u1[m] = d[m + s]
    assert np.allclose(u1, np.roll(d, tuple(-si for si in s), axis=(0, 1, 2)), rtol=1e-13, atol=0)
    u3, _, _ = oracle.rl(d, h, u0, 3)
    assert np.allclose(u3, u1, rtol=1e-13, atol=0)


def test_uniform_psf_closed_form():
    shape = (3, 4, 5)
    d = rng_data(shape, 18)
    u0 = rng_data(shape, 19, 0.5, 2.0)
    h = np.ones(shape)
    K = oracle.otf(h)
    assert np.allclose(oracle.forward(u0, K), np.full(shape, u0.mean()), rtol=1e-13)
    u1, _, _ = oracle.rl(d, h, u0, 1)
    assert np.allclose(u1, u0 * d.sum() / u0.sum(), rtol=1e-13)
    u4, _, _ = oracle.rl(d, h, u0, 4)
    assert np.allclose(u4, u1, rtol=1e-13)


def test_constant_data_is_fixed():
    shape = (4, 5, 6)
    h = rng_psf(shape, 20)
    d = np.full(shape, 7.25)
    u, _, _ = oracle.rl(d, h, d.copy(), 6)
    assert np.allclose(u, d, rtol=1e-13, atol=0)


def test_flux_nonneg_em_and_resume():
    shape = (8, 12, 10)
    h = rng_psf(shape, 21)
    d = np.random.default_rng(22).poisson(30.0, size=shape).astype(float) + 1.0
    u0 = np.full(shape, d.mean())
    u, flux, ll = oracle.rl(d, h, u0, 12, with_loglik=True)
    assert np.all(np.abs(flux - d.sum()) <= 1e-12 * d.sum())
    assert np.all(u >= 0)
    assert np.all(np.diff(ll) >= -1e-12 * np.abs(ll[:-1]))
    ua, _, _ = oracle.rl(d, h, u0, 5)
    ub, _, _ = oracle.rl(d, h, ua, 7)
    assert np.array_equal(ub, u)


def test_zero_data_guard():
    # d = 0 on part of the volume and a PSF with holes: no NaN/Inf; u -> 0 where nothing is seen
    shape = (4, 4, 4)
    h = _delta(shape)
    d = rng_data(shape, 23)
    d[:2] = 0.0
    u0 = np.full(shape, 1.0)
    u, flux, _ = oracle.rl(d, h, u0, 3)
    assert np.all(np.isfinite(u))
    # the DFT of a delta is exact only up to rounding, so "0" means <= 1e-12 of the peak
    assert np.max(np.abs(u[:2])) <= 1e-12 * np.max(u)
    dz = np.zeros(shape)
    u, _, _ = oracle.rl(dz, rng_psf(shape, 24), u0, 2)
    assert np.all(u == 0.0)
    # estimate 0 somewhere: q can vanish; the guard keeps r finite
    u0z = np.zeros(shape)
    u, _, _ = oracle.rl(d, h, u0z, 2)
    assert np.all(u == 0.0)


# --------------------------------------------------------------------------
# Planted mistakes: each plausible error must be caught by one of the pins
# --------------------------------------------------------------------------

def _pins_hold():
    """Re-run a compact set of the pins; False if any fails."""
    try:
        shape = (3, 4, 5)
        h = rng_psf(shape, 30, zero_frac=0.3)
        x = rng_data(shape, 31)
        if not close(rl_oracle.conv3d(x, h), brute_conv(x, h), 1e-10):
            return False
        K = rl_oracle.otf(h)
        if not close(rl_oracle.adjoint(x, K), brute_corr(x, h), 1e-10):
            return False
        rng = np.random.default_rng(32)
        hi = rng.integers(0, 6, size=(2, 3, 4)).astype(float); hi.flat[-1] += 1
        d = rng.integers(1, 20, size=(2, 3, 4)).astype(float)
        u0 = np.full((2, 3, 4), Fraction(int(d.sum()), d.size), dtype=object)
        u, _, _ = rl_oracle.rl(d, hi, u0.astype(float), 2)
        if not close(u, exact_rl(d, hi, u0, 2), 1e-10):
            return False
        return True
    except Exception:
        return False


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


def _mut_flip_adjoint(y, K):
    # "mirrored PSF" taken as an array reversal of the centred kernel's transform
    return np.real(rl_oracle.idft3(K[::-1, ::-1, ::-1] * rl_oracle.dft3(y)))


def _mut_no_conj(y, K):
    return np.real(rl_oracle.idft3(K * rl_oracle.dft3(y)))


def _mut_centre_off(shape):
    return tuple(int(n) // 2 + 1 for n in shape)


def _mut_dft_sign(n, inverse=False):
    # inverse built with the forward sign (a missing conjugation)
    idx = np.arange(n)
    t = np.outer(idx, idx) % n
    ang = 2.0 * np.pi * t / n
    return np.cos(ang) - 1j * np.sin(ang)


def _mut_dft_transposed_phase(n, inverse=False):
    idx = np.arange(n)
    t = np.outer(idx, idx + 1) % n  # wrong index
    ang = 2.0 * np.pi * t / n
    sgn = 1.0 if inverse else -1.0
    return np.cos(ang) + 1j * sgn * np.sin(ang)


def _mut_ratio_inverted(d, q, eps=rl_oracle.EPS):
    ok = q > eps
    return np.where(ok, q / np.where(ok, d, 1.0), 0.0)


def _mut_no_normalise(h):
    hn = np.asarray(h, dtype=np.float64)
    c = rl_oracle.psf_centre(hn.shape)
    return np.roll(hn, shift=tuple(-ci for ci in c), axis=(0, 1, 2))


@pytest.mark.parametrize("name,attr,mut", [
    ("flip instead of adjoint", "adjoint", _mut_flip_adjoint),
    ("adjoint without conj", "adjoint", _mut_no_conj),
    ("centre off by one", "psf_centre", _mut_centre_off),
    ("inverse DFT not conjugated", "dft_matrix", _mut_dft_sign),
    ("wrong DFT phase index", "dft_matrix", _mut_dft_transposed_phase),
    ("ratio inverted", "ratio", _mut_ratio_inverted),
    ("PSF not normalised", "centred_kernel", _mut_no_normalise),
])
def test_planted_mistake_is_caught(monkeypatch, name, attr, mut):
    monkeypatch.setattr(rl_oracle, attr, mut)
    assert not _pins_hold(), name
