"""Pins of the SSIM oracle.

* Brute force: every window's statistics summed voxel by voxel in pure Python on
  a tiny volume (the definition written out), against the cumulative-sum route.
* Identity: SSIM(g, g) = 1; symmetry when the range is fixed; values in [-1, 1].
* The window sums against scipy.ndimage.uniform_filter (an independent library),
  cropped to the valid positions.
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
