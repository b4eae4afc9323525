"""FP64 CPU oracle for the structural similarity index (SSIM).

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it, and it imports nothing from the GPU package.

The paper lists SSIM (Wang et al., 2004) against ground truth among its
deconvolution metrics (§4.3) without parameters.  Reading (the common defaults
of the Python imaging libraries the paper builds on): a uniform 7x7x7 window,
K1 = 0.01, K2 = 0.03, dynamic range L = max(g) - min(g) of the reference, sample
(co)variances (normalised by W - 1, W = 343 voxels), and the mean of the SSIM
map over the voxels whose whole window lies inside the volume:

  S = (2 mu_u mu_g + C1)(2 s_ug + C2) / ((mu_u^2 + mu_g^2 + C1)(s_u^2 + s_g^2 + C2)),
  C1 = (K1 L)^2, C2 = (K2 L)^2.
"""

from __future__ import annotations

import numpy as np

WIN = 7
K1, K2 = 0.01, 0.03


def _window_sums(x: np.ndarray, win: int) -> np.ndarray:
    """Sum over every win^3 window lying inside the volume (valid positions only),
    by cumulative sums along each axis."""
    out = np.asarray(x, dtype=np.float64)
    for ax in range(3):
        c = np.cumsum(out, axis=ax)
        zero = np.zeros_like(np.take(c, [0], axis=ax))
        c = np.concatenate([zero, c], axis=ax)
        n = out.shape[ax]
        out = np.take(c, np.arange(win, n + 1), axis=ax) - np.take(c, np.arange(0, n + 1 - win),
                                                                   axis=ax)
    return out


def ssim(u, g, win: int = WIN, data_range: float | None = None) -> float:
    """Mean SSIM of u against the reference g over the valid window positions."""
    u = np.asarray(u, dtype=np.float64)
    g = np.asarray(g, dtype=np.float64)
    if any(n < win for n in u.shape):
        raise ValueError("every dimension must be at least the window size")
    L = float(g.max() - g.min()) if data_range is None else float(data_range)
    W = float(win ** 3)
    mu_u = _window_sums(u, win) / W
    mu_g = _window_sums(g, win) / W
    cn = W / (W - 1.0)
    vu = cn * (_window_sums(u * u, win) / W - mu_u * mu_u)
    vg = cn * (_window_sums(g * g, win) / W - mu_g * mu_g)
    cug = cn * (_window_sums(u * g, win) / W - mu_u * mu_g)
    c1, c2 = (K1 * L) ** 2, (K2 * L) ** 2
    s = ((2 * mu_u * mu_g + c1) * (2 * cug + c2)) / ((mu_u ** 2 + mu_g ** 2 + c1) * (vu + vg + c2))
    return float(s.mean())
