"""Pins of the SSIM oracle.

* Brute force: every window's statistics summed voxel by voxel in pure Python on
  a tiny volume (the definition written out), against the cumulative-sum route.
* Identity: SSIM(g, g) = 1; symmetry when the range is fixed; values in [-1, 1].
* The window sums against scipy.ndimage.uniform_filter (an independent library),
  cropped to the valid positions.
* A closed form: u = a g + b with constant a > 0 on a volume whose every window
  holds the same sample variance v (a linear ramp), for which each window's SSIM
  is a product of two known factors.
* The last block plants plausible mistakes in the oracle and checks that a pin
  catches each.
"""

import itertools

import numpy as np
from scipy import ndimage

from oracle import ssim_oracle as so


def rng(seed):
    return np.random.default_rng(seed)


def _brute(u, g, win=3, L=None):
    u = np.asarray(u, float)
    g = np.asarray(g, float)
    L = g.max() - g.min() if L is None else L
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    W = win ** 3
    vals = []
    ranges = [range(n - win + 1) for n in u.shape]
    for z, y, x in itertools.product(*ranges):
        a = [u[z + i, y + j, x + k] for i in range(win) for j in range(win) for k in range(win)]
        b = [g[z + i, y + j, x + k] for i in range(win) for j in range(win) for k in range(win)]
        ma, mb = sum(a) / W, sum(b) / W
        va = sum((t - ma) ** 2 for t in a) / (W - 1)
        vb = sum((t - mb) ** 2 for t in b) / (W - 1)
        cab = sum((s - ma) * (t - mb) for s, t in zip(a, b)) / (W - 1)
        vals.append(((2 * ma * mb + c1) * (2 * cab + c2)) /
                    ((ma * ma + mb * mb + c1) * (va + vb + c2)))
    return sum(vals) / len(vals)


def test_brute_force_window_statistics():
    u = rng(1).uniform(0, 10, size=(4, 5, 6))
    g = u + rng(2).normal(0, 1.0, size=u.shape)
    assert abs(so.ssim(u, g, win=3) - _brute(u, g, 3)) <= 1e-12


def test_identity_symmetry_bounds():
    g = rng(3).uniform(0, 100, size=(9, 10, 11))
    u = g + rng(4).normal(0, 10.0, size=g.shape)
    assert abs(so.ssim(g, g) - 1.0) <= 1e-12
    L = 150.0
    assert abs(so.ssim(u, g, data_range=L) - so.ssim(g, u, data_range=L)) <= 1e-12
    assert -1.0 <= so.ssim(u, g) <= 1.0
    assert so.ssim(u, g) < so.ssim(0.5 * (u + g), g)


def test_window_sums_against_uniform_filter():
    x = rng(5).uniform(size=(9, 8, 10))
    w = 7
    ref = ndimage.uniform_filter(x, size=w, mode="constant") * w ** 3
    c = w // 2
    crop = ref[c:x.shape[0] - c, c:x.shape[1] - c, c:x.shape[2] - c]
    assert np.allclose(so._window_sums(x, w), crop, rtol=1e-12, atol=1e-12)


def test_affine_ramp_closed_form():
    # g a linear ramp: every 7^3 window has the same sample variance v and a mean
    # equal to the ramp at its centre; u = a g + b then gives, per window,
    # S = (2 a m^2 + 2 b m + C1)(2 a v + C2) / ((m^2 + (a m + b)^2 + C1)((1 + a^2) v + C2))
    shape = (8, 9, 10)
    z, y, x = np.meshgrid(*[np.arange(n, dtype=float) for n in shape], indexing="ij")
    g = 3.0 * z + 2.0 * y + 1.0 * x + 4.0
    a, b = 0.6, 1.5
    u = a * g + b
    w = so.WIN
    # sample variance of (3i + 2j + k) over i, j, k = 0..w-1, normalised by W - 1
    W = w ** 3
    t = np.arange(w, dtype=float)
    var1 = np.sum((t - t.mean()) ** 2) / w              # per-axis population variance
    v = (9.0 + 4.0 + 1.0) * var1 * W / (W - 1)
    L = g.max() - g.min()
    c1, c2 = (0.01 * L) ** 2, (0.03 * L) ** 2
    c = w // 2
    m = g[c:shape[0] - c, c:shape[1] - c, c:shape[2] - c]
    s = ((2 * m * (a * m + b) + c1) * (2 * a * v + c2)) / \
        ((m * m + (a * m + b) ** 2 + c1) * ((1 + a * a) * v + c2))
    assert abs(so.ssim(u, g) - s.mean()) <= 1e-12


# ---------------------------------------------------------------------------
# Planted mistakes: each must make one of the pins above fail.
# ---------------------------------------------------------------------------
import pytest  # noqa: E402

from mutation import mutate  # noqa: E402


def _pins_hold():
    """Re-run the pins; False if any fails."""
    try:
        for t in (test_brute_force_window_statistics, test_identity_symmetry_bounds,
                  test_window_sums_against_uniform_filter, test_affine_ramp_closed_form):
            t()
    except Exception:
        return False
    return True


def test_pins_hold_on_clean_oracle():
    assert _pins_hold()


@pytest.mark.parametrize("func,old,new", [
    # population instead of sample (co)variances
    ("ssim", "cn = W / (W - 1.0)", "cn = 1.0"),
    # dynamic range of the estimate instead of the reference
    ("ssim", "float(g.max() - g.min())", "float(u.max() - u.min())"),
    ("ssim", "c1, c2 = (K1 * L) ** 2, (K2 * L) ** 2", "c1, c2 = (K2 * L) ** 2, (K1 * L) ** 2"),
    ("ssim", "(2 * cug + c2)", "(cug + c2)"),
    ("ssim", "(vu + vg + c2)", "(vu * vg + c2)"),
    ("ssim", "return float(s.mean())", "return float(np.median(s))"),
    # windows one voxel short
    ("_window_sums", "np.arange(win, n + 1)", "np.arange(win - 1, n)"),
    # the first partial sum in place of the leading zero: windows lose their first plane
    ("_window_sums", "c = np.concatenate([zero, c], axis=ax)",
     "c = np.concatenate([np.take(c, [0], axis=ax), c], axis=ax)"),
])
def test_planted_mistake_is_caught(monkeypatch, func, old, new):
    monkeypatch.setattr(so, func, mutate(so, func, old, new))
    assert not _pins_hold(), (func, new)
