"""FP64 CPU oracle for periodic 3-D Richardson-Lucy deconvolution.

TEST INFRASTRUCTURE. This module is the slow, plainly written reference that
the GPU library is checked against. Only ``tests/``, ``__graft_entry__.smoke()``
and the ``cpu_baseline`` leg of ``bench.py`` may import it. It imports nothing
from the GPU package and the GPU package imports nothing from it.

What is computed (paper §4.3, paragraph "Richardson-Lucy algorithm"): an
iterative deconvolution that maximises the Poisson likelihood; one iteration
blurs the current estimate with the PSF, divides the observed volume by that
blur, blurs the ratio with the mirrored PSF and multiplies the result into the
estimate. This is the EM iteration of Richardson (1972) and Lucy (1974), the
works the paper cites for it (§3.2). The data are ZYX volumes whose PSF has the
image's shape (§4.3, paragraph "Dataset description").

The paper gives no formula, so the following readings are taken (each is
listed with its reason in the design notes of the repository):

* PSF normalised to unit sum in FP64; its centre is voxel floor(n/2) on every
  axis; the convolution is circular (periodic boundary).
* "Mirrored PSF" = the exact adjoint of that circular convolution, i.e. the
  correlation with the centred kernel, which is multiplication by conj(OTF).
* Ratio guard: r = d / q where q > EPS, else 0, with EPS = 1e-12.
* Update clamp: u <- u * max(c, 0) (a no-op in exact arithmetic).

The DFT is applied by its definition: per-axis DFT matrices whose phase index
(j*l) mod n is reduced in exact integer arithmetic, applied with a matrix
product along each axis in turn (the 3-D DFT is separable).  No FFT
factorisation is used.  A second, independent route (``*_direct``) evaluates
the circular convolution and correlation sums by definition.

Parity: pinned by mathematics (convolution theorem vs brute force, an
independent FFT library, adjointness, closed forms, flux conservation,
non-negativity, EM monotonicity, exact rational brute force); the paper prints
no worked RL example, so parity with the paper's own numbers is unpinned.
"""

from __future__ import annotations

import numpy as np

EPS = 1e-12  # ratio guard: q must exceed this for d/q to be taken


# --------------------------------------------------------------------------
# DFT by definition
# --------------------------------------------------------------------------

def dft_matrix(n: int, inverse: bool = False) -> np.ndarray:
    """W[k, j] = exp(-+ 2 pi i (k j mod n) / n); forward sign is negative."""
    idx = np.arange(n, dtype=np.int64)
    t = np.outer(idx, idx) % n            # exact integer phase index
    ang = 2.0 * np.pi * t.astype(np.float64) / n
    sgn = 1.0 if inverse else -1.0
    return np.cos(ang) + 1j * sgn * np.sin(ang)


def _apply_along(x: np.ndarray, w: np.ndarray, axis: int) -> np.ndarray:
    """y[..., k, ...] = sum_j w[k, j] * x[..., j, ...] along ``axis``."""
    xm = np.ascontiguousarray(np.moveaxis(x, axis, -1))
    shp = xm.shape
    ym = np.matmul(xm.reshape(-1, shp[-1]), w.T).reshape(shp)  # one BLAS product
    return np.moveaxis(ym, -1, axis)


def dft3(x: np.ndarray) -> np.ndarray:
    """Forward 3-D DFT, X[k] = sum_m x[m] exp(-2 pi i <k, m/n>)."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(3):
        y = _apply_along(y, dft_matrix(y.shape[ax]), ax)
    return y


def idft3(x: np.ndarray) -> np.ndarray:
    """Inverse 3-D DFT with the 1/N factor."""
    y = np.asarray(x, dtype=np.complex128)
    for ax in range(3):
        y = _apply_along(y, dft_matrix(y.shape[ax], inverse=True), ax)
    return y / float(np.prod(y.shape))


# --------------------------------------------------------------------------
# PSF handling
# --------------------------------------------------------------------------

def psf_centre(shape) -> tuple:
    """Voxel that holds the PSF's peak: floor(n/2) per axis."""
    return tuple(int(n) // 2 for n in shape)


def check_psf(h: np.ndarray) -> float:
    """Return sum(h) in FP64; raise if h is negative, non-finite or sums to <= 0."""
    h64 = np.asarray(h, dtype=np.float64)
    if not np.all(np.isfinite(h64)):
        raise ValueError("PSF has non-finite entries")
    if np.any(h64 < 0):
        raise ValueError("PSF has negative entries")
    s = float(h64.sum())
    if not s > 0.0:
        raise ValueError("PSF sums to zero")
    return s


def centred_kernel(h: np.ndarray) -> np.ndarray:
    """k[m] = (h / sum h)[(m + c) mod n]: unit-sum PSF with its centre moved to 0."""
    s = check_psf(h)
    hn = np.asarray(h, dtype=np.float64) / s
    c = psf_centre(hn.shape)
    return np.roll(hn, shift=tuple(-ci for ci in c), axis=(0, 1, 2))


def otf(h: np.ndarray) -> np.ndarray:
    """Transfer function K = DFT(k) of the centred, normalised kernel."""
    return dft3(centred_kernel(h))


# --------------------------------------------------------------------------
# Forward operator H and its adjoint
# --------------------------------------------------------------------------

def forward(x: np.ndarray, K: np.ndarray) -> np.ndarray:
    """H x = Re IDFT(K * DFT x): circular convolution with the PSF."""
    return np.real(idft3(K * dft3(x)))


def adjoint(y: np.ndarray, K: np.ndarray) -> np.ndarray:
    """H^T y = Re IDFT(conj(K) * DFT y): circular correlation with the PSF."""
    return np.real(idft3(np.conj(K) * dft3(y)))


def conv3d(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """The forward operator applied to x, built from the raw PSF h."""
    return forward(np.asarray(x, dtype=np.float64), otf(h))


# Direct sums (independent of the DFT route) --------------------------------

def conv_direct(x: np.ndarray, h: np.ndarray) -> np.ndarray:
    """(H x)[m] = sum_j k[j] x[(m - j) mod n], summed over every j with k[j] != 0."""
    k = centred_kernel(h)
    x = np.asarray(x, dtype=np.float64)
    out = np.zeros_like(x)
    for j in zip(*np.nonzero(k)):
        out += k[j] * np.roll(x, shift=j, axis=(0, 1, 2))
    return out


def corr_direct(y: np.ndarray, h: np.ndarray) -> np.ndarray:
    """(H^T y)[m] = sum_j k[j] y[(m + j) mod n]."""
    k = centred_kernel(h)
    y = np.asarray(y, dtype=np.float64)
    out = np.zeros_like(y)
    for j in zip(*np.nonzero(k)):
        out += k[j] * np.roll(y, shift=tuple(-ji for ji in j), axis=(0, 1, 2))
    return out


def conv_direct_at(x: np.ndarray, h: np.ndarray, points) -> np.ndarray:
    """(H x)[m] for each voxel m in ``points`` by the direct sum over all N voxels."""
    k = centred_kernel(h)
    x = np.asarray(x, dtype=np.float64)
    nz, ny, nx = x.shape
    jz, jy, jx = np.arange(nz), np.arange(ny), np.arange(nx)
    out = []
    for (mz, my, mx) in points:
        xs = x[np.ix_((mz - jz) % nz, (my - jy) % ny, (mx - jx) % nx)]
        out.append(float(np.sum(k * xs)))
    return np.array(out)


# --------------------------------------------------------------------------
# Richardson-Lucy
# --------------------------------------------------------------------------

def ratio(d: np.ndarray, q: np.ndarray, eps: float = EPS) -> np.ndarray:
    """r = d / q where q > eps, else 0."""
    ok = q > eps
    return np.where(ok, d / np.where(ok, q, 1.0), 0.0)


def loglik(d: np.ndarray, q: np.ndarray, eps: float = EPS) -> float:
    """Poisson log-likelihood up to a constant, over voxels with q > eps."""
    ok = q > eps
    dd, qq = d[ok], q[ok]
    pos = dd > 0
    return float(np.sum(dd[pos] * np.log(qq[pos])) - np.sum(qq))


def rl(d, h, u0, n_iter: int, eps: float = EPS, with_loglik: bool = False):
    """Run ``n_iter`` Richardson-Lucy iterations from u0.

    Returns (u, flux, ll): the FP64 estimate after n_iter iterations, the total
    flux sum(u_t) after each iteration t = 1..n_iter, and (when requested) the
    log-likelihood of u_t for t = 0..n_iter-1, evaluated at q = H u_t.
    """
    if n_iter < 0:
        raise ValueError("n_iter must be >= 0")
    d = np.asarray(d, dtype=np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    K = otf(h)
    flux, ll = [], []
    for _ in range(n_iter):
        q = forward(u, K)
        if with_loglik:
            ll.append(loglik(d, q, eps))
        r = ratio(d, q, eps)
        c = adjoint(r, K)
        u = u * np.maximum(c, 0.0)
        flux.append(float(u.sum()))
    return u, np.array(flux), np.array(ll)


def rl_direct(d, h, u0, n_iter: int, eps: float = EPS):
    """Richardson-Lucy with both blurs evaluated by their direct sums."""
    d = np.asarray(d, dtype=np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    for _ in range(n_iter):
        q = conv_direct(u, h)
        r = ratio(d, q, eps)
        c = corr_direct(r, h)
        u = u * np.maximum(c, 0.0)
    return u


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 in FP64 (b is the reference)."""
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    nb = float(np.linalg.norm(b.ravel()))
    na = float(np.linalg.norm((a - b).ravel()))
    return na / nb if nb > 0 else na
