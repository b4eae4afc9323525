"""FP64 CPU oracle for PSFs smaller than the volume and for the zero boundary.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it, and it imports nothing from the GPU package.

PSF of any shape p <= n per axis.  Its centre is voxel c = floor(p/2) per axis
and its weights are normalised to unit sum in FP64 (as for a PSF of the
image's shape, paper §4.3 "Dataset description"); entry m sits at offset
k = m - c from the centre.

* Periodic boundary: (H x)[i] = sum_m h^[m] x[(i - (m - c)) mod n], the circular
  convolution with the PSF embedded, centred, in the volume's grid.
* Zero boundary: the same sum with x taken as zero outside the volume (linear
  convolution, the volume's own grid kept: the "same"-size output of a
  zero-padded convolution).  Its adjoint is
  (H^T y)[i] = sum_m h^[m] y[i + (m - c)], y zero outside the volume.

Richardson-Lucy then runs unchanged on either operator:
u <- u * max(H^T (d / H u), 0) with the ratio guard of ``rl_oracle``.  No
normalisation by H^T 1 is applied at the borders (reading: the zero boundary
keeps the plain update, as the scikit-image routine that the paper's library
exposes does); the total flux is still conserved, since
sum_j u_j (H^T r)_j = sum_i r_i (H u)_i = sum_{q>eps} d_i for any H.

Routes: the DFT route (embed, circular convolution on a grid large enough that
no wrapped term reaches the volume, crop) and a direct route (one shifted,
cropped copy of x per PSF entry).  Pinned against an independent library
(scipy.signal's full linear convolution), against the pinned same-shape
periodic oracle, by brute-force sums and by adjointness.
"""

from __future__ import annotations

import numpy as np

from .rl_oracle import EPS, check_psf, dft3, idft3, psf_centre, ratio


def _normalised(h) -> np.ndarray:
    return np.asarray(h, dtype=np.float64) / check_psf(h)


def embed_kernel(h, shape) -> np.ndarray:
    """Unit-sum PSF placed on a grid of `shape` with offset k at index k mod n."""
    hn = _normalised(h)
    if any(p > n for p, n in zip(hn.shape, shape)):
        raise ValueError("PSF larger than the grid")
    c = psf_centre(hn.shape)
    out = np.zeros(tuple(int(n) for n in shape))
    idx = [((np.arange(p) - ci) % n) for p, ci, n in zip(hn.shape, c, shape)]
    out[np.ix_(*idx)] = hn
    return out


def conv_periodic(x, h) -> np.ndarray:
    """Circular convolution of x with the (possibly smaller) PSF h."""
    x = np.asarray(x, dtype=np.float64)
    K = dft3(embed_kernel(h, x.shape))
    return np.real(idft3(K * dft3(x)))


def corr_periodic(y, h) -> np.ndarray:
    """Adjoint of conv_periodic."""
    y = np.asarray(y, dtype=np.float64)
    K = dft3(embed_kernel(h, y.shape))
    return np.real(idft3(np.conj(K) * dft3(y)))


def _padded_grid(shape, psf_shape, extra: int = 0) -> tuple:
    # n + p - 1 per axis: no wrapped term of a circular convolution on this grid
    # reaches indices [0, n) from outside them
    return tuple(int(n) + int(p) - 1 + extra for n, p in zip(shape, psf_shape))


def _embed(x, grid) -> np.ndarray:
    out = np.zeros(grid)
    out[tuple(slice(0, n) for n in x.shape)] = x
    return out


def conv_zero(x, h, extra_pad: int = 0) -> np.ndarray:
    """Linear convolution with the PSF, x zero outside the volume, cropped to it."""
    x = np.asarray(x, dtype=np.float64)
    grid = _padded_grid(x.shape, np.shape(h), extra_pad)
    K = dft3(embed_kernel(h, grid))
    full = np.real(idft3(K * dft3(_embed(x, grid))))
    return full[tuple(slice(0, n) for n in x.shape)]


def corr_zero(y, h, extra_pad: int = 0) -> np.ndarray:
    """Adjoint of conv_zero: linear correlation, y zero outside the volume."""
    y = np.asarray(y, dtype=np.float64)
    grid = _padded_grid(y.shape, np.shape(h), extra_pad)
    K = dft3(embed_kernel(h, grid))
    full = np.real(idft3(np.conj(K) * dft3(_embed(y, grid))))
    return full[tuple(slice(0, n) for n in y.shape)]


def _shifted(x, k) -> np.ndarray:
    """s[i] = x[i - k] where i - k lies inside the volume, else 0."""
    out = np.zeros_like(x)
    dst, src = [], []
    for ki, n in zip(k, x.shape):
        lo, hi = max(0, ki), min(n, n + ki)
        if lo >= hi:
            return out
        dst.append(slice(lo, hi))
        src.append(slice(lo - ki, hi - ki))
    out[tuple(dst)] = x[tuple(src)]
    return out


def conv_zero_direct(x, h) -> np.ndarray:
    """Direct route of conv_zero: one shifted copy of x per non-zero PSF entry."""
    x = np.asarray(x, dtype=np.float64)
    hn = _normalised(h)
    c = psf_centre(hn.shape)
    out = np.zeros_like(x)
    for m in zip(*np.nonzero(hn)):
        out += hn[m] * _shifted(x, tuple(mi - ci for mi, ci in zip(m, c)))
    return out


def corr_zero_direct(y, h) -> np.ndarray:
    """Direct route of corr_zero."""
    y = np.asarray(y, dtype=np.float64)
    hn = _normalised(h)
    c = psf_centre(hn.shape)
    out = np.zeros_like(y)
    for m in zip(*np.nonzero(hn)):
        out += hn[m] * _shifted(y, tuple(ci - mi for mi, ci in zip(m, c)))
    return out


def conv_zero_at(x, h, points) -> np.ndarray:
    """conv_zero(x, h)[m] for each voxel m in ``points``, by the direct sum over the
    PSF entries whose shifted voxel lies inside the volume."""
    x = np.asarray(x, dtype=np.float64)
    hn = _normalised(h)
    c = psf_centre(hn.shape)
    out = []
    for m in points:
        idx, keep = [], []
        for ax in range(3):
            j = np.arange(hn.shape[ax])
            src = m[ax] - (j - c[ax])
            ok = (src >= 0) & (src < x.shape[ax])
            idx.append(src[ok])
            keep.append(j[ok])
        out.append(float(np.sum(hn[np.ix_(*keep)] * x[np.ix_(*idx)])))
    return np.array(out)


def operators(h, boundary: str):
    """(H, H^T) as functions of a volume, for boundary 'periodic' or 'zero'."""
    if boundary == "periodic":
        return (lambda x: conv_periodic(x, h)), (lambda y: corr_periodic(y, h))
    if boundary == "zero":
        return (lambda x: conv_zero(x, h)), (lambda y: corr_zero(y, h))
    raise ValueError("boundary must be 'periodic' or 'zero'")


def rl_general(d, h, u0, n_iter: int, boundary: str = "periodic", eps: float = EPS):
    """Richardson-Lucy with a PSF of any shape <= the volume and either boundary.

    Returns (u, flux) like ``rl_oracle.rl`` (flux = sum(u_t) after each iteration).
    """
    if n_iter < 0:
        raise ValueError("n_iter must be >= 0")
    fwd, adj = operators(h, boundary)
    d = np.asarray(d, dtype=np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    flux = []
    for _ in range(n_iter):
        u = u * np.maximum(adj(ratio(d, fwd(u), eps)), 0.0)
        flux.append(float(u.sum()))
    return u, np.array(flux)
