"""Pins of the FSC oracle.

* Identity and sign: FSC(a, a) = 1, FSC(a, -a) = -1, FSC(a, c a) = 1 in every
  shell that holds energy.
* Parseval: the |F|^2 sums over all shells (corners included) equal N sum a^2.
* A closed form: for a single spatial frequency k0 and b = a shifted by s
  voxels, all energy sits in the shell of k0 and the FSC there is
  cos(2 pi k0 . s / n).
* The shell map against numpy.fft.fftfreq (an independent library).
* The resolution crossing on hand-made curves; shell 0 never counts as a crossing.
* The last block plants plausible mistakes in the oracle and checks that a pin
  catches each.
"""

import numpy as np
import pytest

from oracle import fsc_oracle as fo


def rng(seed):
    return np.random.default_rng(seed)


@pytest.mark.parametrize("shape", [(6, 8, 10), (5, 7, 9), (1, 12, 16)])
def test_identity_sign_scale(shape):
    a = rng(1).normal(size=shape)
    nb = 6
    num, d1, _ = fo.fsc_sums(a, a, nb)
    live = d1 > 0
    assert np.allclose(fo.fsc(a, a, nb)[live], 1.0, atol=1e-12)
    assert np.allclose(fo.fsc(a, -a, nb)[live], -1.0, atol=1e-12)
    assert np.allclose(fo.fsc(a, 3.5 * a, nb)[live], 1.0, atol=1e-12)


def test_parseval():
    a = rng(2).normal(size=(6, 8, 10))
    _, d1, _ = fo.fsc_sums(a, a, 5)
    assert abs(d1.sum() - a.size * np.sum(a * a)) <= 1e-9 * a.size * np.sum(a * a)


def test_single_frequency_shift_closed_form():
    shape = (8, 12, 16)
    k0 = np.array([1, 2, 3])
    s = np.array([0, 1, 2])
    idx = np.meshgrid(*[np.arange(n) for n in shape], indexing="ij")
    phase = sum(2 * np.pi * k0[i] * idx[i] / shape[i] for i in range(3))
    a = np.cos(phase)
    b = np.roll(a, shift=tuple(s), axis=(0, 1, 2))
    nb = 8
    curve = fo.fsc(a, b, nb)
    _, d1, _ = fo.fsc_sums(a, b, nb)
    shell = int(np.floor(np.sqrt(np.sum((k0 / np.array(shape)) ** 2)) / 0.5 * nb))
    assert np.count_nonzero(d1 > 1e-9) == 1 and d1[shell] > 0
    want = np.cos(2 * np.pi * np.sum(k0 * s / np.array(shape)))
    assert abs(curve[shell] - want) <= 1e-12


def test_shell_map_against_fftfreq():
    shape = (5, 8, 7)
    nb = 10
    fz, fy, fx = np.meshgrid(*[np.fft.fftfreq(n) for n in shape], indexing="ij")
    rho = np.sqrt(fz ** 2 + fy ** 2 + fx ** 2)
    want = np.minimum(np.floor(rho / 0.5 * nb).astype(int), nb)
    assert np.array_equal(fo.shell_index(shape, nb), want)


def test_resolution_crossing():
    nb = 10
    f = (np.arange(nb) + 0.5) * 0.05
    curve = np.array([1.0, 0.9, 0.8, 0.5, 0.3, 0.1, 0.05, 0.0, 0.0, 0.0])
    # crossing of 1/7 between shells 4 (0.3) and 5 (0.1)
    t = (0.3 - 1 / 7) / (0.3 - 0.1)
    assert abs(fo.resolution(curve, nb) - (f[4] + t * (f[5] - f[4]))) <= 1e-15
    assert fo.resolution(np.ones(nb), nb) == 0.5
    assert abs(fo.resolution(curve, nb, threshold=0.85) - (f[1] + 0.5 * (f[2] - f[1]))) <= 1e-15


def test_split_diagonal():
    u = np.arange(4 * 6 * 8, dtype=float).reshape(4, 6, 8)
    a, b = fo.split_diagonal(u)
    assert a.shape == (2, 3, 4) and b.shape == (2, 3, 4)
    assert a[1, 2, 3] == u[2, 4, 6] and b[1, 2, 3] == u[3, 5, 7]


def test_dc_shell_is_not_a_crossing():
    # shell 0 holds the mean; a low value there is not a resolution crossing
    nb = 8
    f = (np.arange(nb) + 0.5) * 0.5 / nb
    curve = np.array([0.0, 0.9, 0.05, 0.0, 0.0, 0.0, 0.0, 0.0])
    t = (0.9 - 1 / 7) / (0.9 - 0.05)
    assert abs(fo.resolution(curve, nb) - (f[1] + t * (f[2] - f[1]))) <= 1e-15


# ---------------------------------------------------------------------------
# Planted mistakes: each must make one of the pins above fail.
# ---------------------------------------------------------------------------
from mutation import mutate  # noqa: E402


def _pins_hold():
    """Re-run a compact set of the pins; False if any fails."""
    tests = [lambda: test_identity_sign_scale((5, 7, 9)), test_parseval,
             test_single_frequency_shift_closed_form, test_shell_map_against_fftfreq,
             test_resolution_crossing, test_dc_shell_is_not_a_crossing, test_split_diagonal]
    try:
        for t in tests:
            t()
    except Exception:
        return False
    return True


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("func,old,new", [
    # unsigned frequency index: the upper half of each axis lands in far shells
    ("signed_index", "j < (n + 1) // 2, j, j - n", "j < n, j, j - n"),
    # shells twice as wide (rho * nbins)
    ("shell_index", "four = 4 * nbins * nbins", "four = nbins * nbins"),
    # a frequency on a shell boundary put into the inner shell
    ("shell_index", "math.isqrt((four * int(v)) // (L * L))",
     "math.isqrt(max((four * int(v) - 1) // (L * L), 0))"),
    ("fsc_sums", "np.real(F * np.conj(G))", "np.real(F * G)"),
    ("fsc_sums", "np.real(F * np.conj(G))", "np.imag(F * np.conj(G))"),
    ("fsc_sums", "(np.abs(G) ** 2)", "(np.abs(F) ** 2)"),
    ("fsc", "np.sqrt(d1 * d2)", "0.5 * (d1 + d2)"),
    ("resolution", "range(1, nbins)", "range(0, nbins)"),
    ("resolution", "f[s - 1] + t * (f[s] - f[s - 1])", "f[s]"),
    ("resolution", "(np.arange(nbins) + 0.5)", "np.arange(nbins)"),
    ("split_diagonal", "u[1::2, 1::2, 1::2]", "u[1::2, 1::2, 0::2]"),
])
def test_planted_mistake_is_caught(monkeypatch, func, old, new):
    monkeypatch.setattr(fo, func, mutate(fo, func, old, new))
    assert not _pins_hold(), (func, new)
