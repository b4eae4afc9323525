"""FP64 CPU oracle for Fourier shell correlation and its single-image split.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it, and it imports nothing from the GPU package.

The paper evaluates deconvolution with a resolution derived from single-image
Fourier ring correlation and lists FRC/FSC among its metrics (§3 and §4.3,
citing Nieuwenhuizen et al. 2013, Banterle et al. 2013 and Koho et al. 2019),
without formulas.  Definitions taken here (readings, listed in the design
notes):

* FSC of volumes a, b (same shape): with F = DFT(a), G = DFT(b) and the
  normalised radius rho(k) = sqrt(sum_i (k_i / n_i)^2) of each frequency, k_i
  the signed index in [-n_i/2, n_i/2), shell s = floor(rho / 0.5 * nbins)
  evaluated exactly (rho^2 is rational; frequencies on a shell boundary belong
  to the outer shell), shells 0 .. nbins-1 covering rho < 0.5 cycles per voxel
  and shell nbins the corners beyond; FSC_s = sum_s Re(F conj G) /
  sqrt(sum_s |F|^2 sum_s |G|^2) (0 where a denominator vanishes).
* Resolution: the first shell s >= 1 with FSC_s below the threshold (default
  1/7); the crossing frequency is interpolated linearly between the centres
  f_s = (s + 0.5) * 0.5 / nbins of shells s-1 and s; 0.5 if the curve never
  drops below it.
* Single-image split: the two diagonal sub-volumes u[0::2, 0::2, 0::2] and
  u[1::2, 1::2, 1::2] (even dimensions).
"""

from __future__ import annotations

import math

import numpy as np

from .rl_oracle import dft3


def signed_index(n: int) -> np.ndarray:
    """k for DFT bin j of length n: j for j < ceil(n/2), j - n after."""
    j = np.arange(n)
    return np.where(j < (n + 1) // 2, j, j - n)


def shell_index(shape, nbins: int) -> np.ndarray:
    """Shell of every frequency of a full DFT grid of `shape`:
    floor(2 nbins rho) = isqrt(floor(4 nbins^2 rho^2)), in exact integer
    arithmetic over the common denominator L = lcm(n_z, n_y, n_x)."""
    L = math.lcm(*[int(n) for n in shape])
    kz, ky, kx = (signed_index(n).astype(object) * (L // n) for n in shape)
    q = (kz[:, None, None] ** 2 + ky[None, :, None] ** 2) + kx[None, None, :] ** 2
    four = 4 * nbins * nbins
    s = np.vectorize(lambda v: math.isqrt((four * int(v)) // (L * L)), otypes=[np.int64])(q)
    return np.minimum(s, nbins)


def fsc_sums(a, b, nbins: int):
    """Per shell (nbins + 1 of them): sum Re(F conj G), sum |F|^2, sum |G|^2."""
    F = dft3(np.asarray(a, dtype=np.float64))
    G = dft3(np.asarray(b, dtype=np.float64))
    s = shell_index(np.shape(a), nbins).ravel()
    num = np.bincount(s, weights=np.real(F * np.conj(G)).ravel(), minlength=nbins + 1)
    d1 = np.bincount(s, weights=(np.abs(F) ** 2).ravel(), minlength=nbins + 1)
    d2 = np.bincount(s, weights=(np.abs(G) ** 2).ravel(), minlength=nbins + 1)
    return num, d1, d2


def fsc(a, b, nbins: int) -> np.ndarray:
    """FSC curve over shells 0 .. nbins (the last one: corners beyond 0.5)."""
    num, d1, d2 = fsc_sums(a, b, nbins)
    den = np.sqrt(d1 * d2)
    return np.where(den > 0, num / np.where(den > 0, den, 1.0), 0.0)


def resolution(curve, nbins: int, threshold: float = 1.0 / 7.0) -> float:
    """Frequency (cycles per voxel) where the curve first drops below threshold."""
    f = (np.arange(nbins) + 0.5) * 0.5 / nbins
    for s in range(1, nbins):
        if curve[s] < threshold:
            c0, c1 = curve[s - 1], curve[s]
            t = (c0 - threshold) / (c0 - c1) if c0 != c1 else 0.0
            return float(f[s - 1] + t * (f[s] - f[s - 1]))
    return 0.5


def split_diagonal(u):
    """The two diagonal sub-volumes of the single-image split."""
    u = np.asarray(u)
    return u[0::2, 0::2, 0::2], u[1::2, 1::2, 1::2]
