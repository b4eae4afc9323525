"""Seeded synthetic microscopy volumes that stand in for the paper's data.

The paper's Richardson-Lucy experiment uses one confocal stack of stained
nuclei with a modelled PSF of the same ZYX size (§4.3, paragraph "Dataset
description"); neither is available, so these generators draw volumes of the
same kind: ellipsoidal nuclei (and point sources) on a background, blurred by an
anisotropic Gaussian PSF that fills the whole grid, with Poisson (and read)
noise.  Every array is C-ordered [Z][Y][X] float32.

This module only draws inputs.  It is shared by the tests, the benchmark and the
oracle checks, and contains none of the deconvolution: the blur that simulates
image formation here uses numpy's FFT and exists only to make realistic input
data; neither the GPU library nor the oracle calls it.

Sizes and distributions (Z, Y, X):
  config 0  (32, 64, 64)    40 Gaussian nuclei + 20 points, PSF sigma (x,y,z)=(1.5,1.5,3)
  config 1  (128, 256, 256) 400 textured solid nuclei, PSF (2,2,5), peak ~2000
  config 2  (256, 512, 512) 3000 nuclei on a spherical shell, PSF (2.5,2.5,6), + read noise
  batch     96 volumes (s/2, s, s), s in {48, 64, 96, 128, 192}, per-volume PSF
  paper     (30, 2160, 2560) the shape of the paper's own stack: 8000 textured
            nuclei (semi-axes x, y in [6, 14], z in [2, 5]), PSF (2, 2, 2.5),
            peak ~2000 photons on background 50, Poisson noise
"""

from __future__ import annotations

import numpy as np

BASE_SEED = 14143
BATCH_SEED = 14147
BATCH_SIDES = (48, 64, 96, 128, 192)

CONFIGS = {
    0: dict(shape=(32, 64, 64), sigma=(1.5, 1.5, 3.0), n_iter=20),
    1: dict(shape=(128, 256, 256), sigma=(2.0, 2.0, 5.0), n_iter=100),
    2: dict(shape=(256, 512, 512), sigma=(2.5, 2.5, 6.0), n_iter=50),
}


def gaussian_psf(shape, sigma_xyz) -> np.ndarray:
    """Point-sampled exp(-1/2 sum (d_i/s_i)^2) over the whole grid, peak at floor(n/2),
    normalised to unit sum in FP64 and stored as float32."""
    nz, ny, nx = shape
    sx, sy, sz = sigma_xyz
    z = (np.arange(nz) - nz // 2) / sz
    y = (np.arange(ny) - ny // 2) / sy
    x = (np.arange(nx) - nx // 2) / sx
    g = (np.exp(-0.5 * z * z)[:, None, None] * np.exp(-0.5 * y * y)[None, :, None]
         * np.exp(-0.5 * x * x)[None, None, :])
    g /= g.sum()
    return g.astype(np.float32)


def _image_formation_blur(vol: np.ndarray, psf: np.ndarray) -> np.ndarray:
    """Periodic blur used only to simulate the microscope when making inputs."""
    k = np.fft.ifftshift(psf.astype(np.float64))
    out = np.fft.irfftn(np.fft.rfftn(vol) * np.fft.rfftn(k), s=vol.shape, axes=(0, 1, 2))
    return np.maximum(out, 0.0)


def _place(rng, shape, semi, centre_fn=None, max_tries=1000):
    """Draw an integer centre such that the box of half-size ``semi`` fits."""
    for _ in range(max_tries):
        if centre_fn is None:
            c = [rng.uniform(semi[i], shape[i] - 1 - semi[i]) for i in range(3)]
        else:
            c = centre_fn(rng)
        if all(semi[i] <= c[i] <= shape[i] - 1 - semi[i] for i in range(3)):
            return c
    raise RuntimeError("could not place object inside the volume")


def _add_gaussian_nucleus(vol, c, a, amp, trunc=1.5):
    """amp * exp(-2 rho^2) with rho the ellipsoidal radius over semi-axes a, rho <= trunc."""
    lo = [max(0, int(np.floor(c[i] - trunc * a[i]))) for i in range(3)]
    hi = [min(vol.shape[i], int(np.ceil(c[i] + trunc * a[i])) + 1) for i in range(3)]
    zz, yy, xx = np.meshgrid(*[np.arange(lo[i], hi[i]) for i in range(3)], indexing="ij")
    rho2 = ((zz - c[0]) / a[0]) ** 2 + ((yy - c[1]) / a[1]) ** 2 + ((xx - c[2]) / a[2]) ** 2
    val = amp * np.exp(-2.0 * rho2) * (rho2 <= trunc * trunc)
    vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += val


def _add_solid_nucleus(vol, rng, c, a, amp, texture=0.2):
    """Solid ellipsoid of value amp * max(0, 1 + texture * xi), xi ~ N(0,1) per voxel."""
    lo = [max(0, int(np.floor(c[i] - a[i]))) for i in range(3)]
    hi = [min(vol.shape[i], int(np.ceil(c[i] + a[i])) + 1) for i in range(3)]
    zz, yy, xx = np.meshgrid(*[np.arange(lo[i], hi[i]) for i in range(3)], indexing="ij")
    rho2 = ((zz - c[0]) / a[0]) ** 2 + ((yy - c[1]) / a[1]) ** 2 + ((xx - c[2]) / a[2]) ** 2
    tex = np.maximum(0.0, 1.0 + texture * rng.standard_normal(rho2.shape))
    vol[lo[0]:hi[0], lo[1]:hi[1], lo[2]:hi[2]] += amp * tex * (rho2 <= 1.0)


def _semi_zyx(rng, lo, hi):
    # semi-axes drawn independently per axis, returned in (z, y, x) order
    ax, ay, az = rng.uniform(lo, hi, size=3)
    return (az, ay, ax)


def gaussian_nuclei_volume(rng, shape, sigma_xyz, n_nuclei, n_points, background=10.0):
    """Config-0 style content: Gaussian nuclei and point sources, Poisson noise."""
    truth = np.zeros(shape, dtype=np.float64)
    for _ in range(n_nuclei):
        a = _semi_zyx(rng, 3.0, 8.0)
        a = tuple(min(a[i], (shape[i] - 1) / 3.0) for i in range(3))
        c = _place(rng, shape, [1.5 * ai for ai in a])
        _add_gaussian_nucleus(truth, c, a, rng.uniform(200.0, 1000.0))
    for _ in range(n_points):
        p = tuple(int(rng.integers(0, shape[i])) for i in range(3))
        truth[p] += rng.uniform(200.0, 1000.0)
    truth += background
    psf = gaussian_psf(shape, sigma_xyz)
    blur = _image_formation_blur(truth, psf)
    d = rng.poisson(blur).astype(np.float32)
    return d, psf, truth


def _solid_nuclei_volume(rng, shape, sigma_xyz, n_nuclei, background, peak,
                         centre_fn=None, read_noise=0.0):
    truth = np.zeros(shape, dtype=np.float64)
    for _ in range(n_nuclei):
        a = _semi_zyx(rng, 4.0, 12.0)
        c = _place(rng, shape, a, centre_fn)
        _add_solid_nucleus(truth, rng, c, a, rng.uniform(200.0, 1000.0))
    psf = gaussian_psf(shape, sigma_xyz)
    blur = _image_formation_blur(truth, psf)
    scale = (peak - background) / max(float(blur.max()), 1e-30)
    lam = blur * scale + background
    d = rng.poisson(lam).astype(np.float64)
    if read_noise > 0:
        d = np.maximum(0.0, d + rng.normal(0.0, read_noise, size=shape))
    return d.astype(np.float32), psf, truth * scale + background


PAPER_SHAPE = (30, 2160, 2560)
PAPER_SIGMA = (2.0, 2.0, 2.5)
PAPER_SEED = 2160


def make_paper_shape(seed: int = PAPER_SEED) -> dict:
    """A volume of the paper's stack shape (Z, Y, X) = (30, 2160, 2560): a flat,
    wide field of textured nuclei, PSF of the volume's shape, Poisson noise.  Built
    in float32 with scipy's multithreaded FFT for the image-formation blur, since
    the volume has 1.7e8 voxels."""
    import os

    import scipy.fft as sfft

    rng = np.random.default_rng(seed)
    shape = PAPER_SHAPE
    truth = np.zeros(shape, dtype=np.float32)
    for _ in range(8000):
        ax, ay = rng.uniform(6.0, 14.0, size=2)
        az = rng.uniform(2.0, 5.0)
        a = (az, ay, ax)
        c = _place(rng, shape, a)
        _add_solid_nucleus(truth, rng, c, a, rng.uniform(200.0, 1000.0))
    # the Gaussian PSF is a product of per-axis factors: normalise each in FP64
    sx, sy, sz = PAPER_SIGMA
    g = []
    for n, sg in zip(shape, (sz, sy, sx)):
        t = (np.arange(n) - n // 2) / sg
        e = np.exp(-0.5 * t * t)
        g.append(e / e.sum())
    gzy = g[0][:, None] * g[1][None, :]
    psf = np.empty(shape, dtype=np.float32)
    for z in range(shape[0]):
        psf[z] = (gzy[z][:, None] * g[2][None, :]).astype(np.float32)
    w = os.cpu_count() or 1
    k = np.fft.ifftshift(psf)
    blur = sfft.irfftn(sfft.rfftn(truth, workers=w) * sfft.rfftn(k, workers=w), s=shape,
                       workers=w)
    del k
    np.maximum(blur, 0.0, out=blur)
    scale = (2000.0 - 50.0) / max(float(blur.max()), 1e-30)
    blur *= np.float32(scale)
    blur += np.float32(50.0)
    d = rng.poisson(blur).astype(np.float32)
    return dict(shape=shape, sigma=PAPER_SIGMA, d=d, psf=psf, u0=initial_estimate(d))


def initial_estimate(d: np.ndarray) -> np.ndarray:
    """u0 = mean(d) everywhere (FP64 mean, stored float32)."""
    return np.full(d.shape, np.float32(np.mean(d, dtype=np.float64)), dtype=np.float32)


def make_config(cfg: int) -> dict:
    """Inputs of benchmark configuration 0, 1 or 2 (3 shares config 2's inputs)."""
    if cfg == 3:
        cfg = 2
    spec = CONFIGS[cfg]
    rng = np.random.default_rng(BASE_SEED + cfg)
    shape, sigma = spec["shape"], spec["sigma"]
    if cfg == 0:
        d, psf, truth = gaussian_nuclei_volume(rng, shape, sigma, 40, 20, background=10.0)
    elif cfg == 1:
        d, psf, truth = _solid_nuclei_volume(rng, shape, sigma, 400, 50.0, 2000.0)
    else:
        nz, ny, nx = shape
        ctr = np.array([nz // 2, ny // 2, nx // 2], dtype=np.float64)

        def on_shell(r):
            v = r.standard_normal(3)
            v /= np.linalg.norm(v)
            return list(ctr + v * (180.0 + r.uniform(-10.0, 10.0)))

        d, psf, truth = _solid_nuclei_volume(rng, shape, sigma, 3000, 50.0, 2000.0,
                                             centre_fn=on_shell, read_noise=3.0)
    return dict(cfg=cfg, shape=shape, sigma=sigma, n_iter=spec["n_iter"], d=d, psf=psf,
                u0=initial_estimate(d), truth=truth.astype(np.float32))


def uniform_volume(shape, seed: int) -> np.ndarray:
    """U(0,1) float32 volume, used as a second convolution input."""
    return np.random.default_rng(seed).uniform(0.0, 1.0, size=shape).astype(np.float32)


def small_case(shape, sigma_xyz=(1.5, 1.5, 3.0), seed: int = 0, density=1.0):
    """Config-0 style content at any shape (nuclei count scaled by volume)."""
    rng = np.random.default_rng(seed)
    n = int(np.prod(shape))
    nn = max(1, int(round(40 * density * n / 131072)))
    npt = max(1, int(round(20 * density * n / 131072)))
    d, psf, truth = gaussian_nuclei_volume(rng, shape, sigma_xyz, nn, npt, background=10.0)
    return dict(shape=tuple(shape), d=d, psf=psf, u0=initial_estimate(d), truth=truth)


def batch_shapes(count: int = 96, seed: int = BATCH_SEED):
    """(Z, Y, X) = (s/2, s, s) with s drawn uniformly from the side set, one per volume."""
    rng = np.random.default_rng(seed)
    sides = rng.choice(np.array(BATCH_SIDES), size=count)
    return [(int(s) // 2, int(s), int(s)) for s in sides]


def make_batch(count: int = 96, seed: int = BATCH_SEED):
    """Batched-form inputs: uneven volumes, each with its own Gaussian PSF."""
    shapes = batch_shapes(count, seed)
    children = np.random.SeedSequence(seed).spawn(count)
    out = []
    for shape, child in zip(shapes, children):
        rng = np.random.default_rng(child)
        sxy = rng.uniform(1.0, 3.0)
        sz = rng.uniform(2.0, 6.0)
        n = int(np.prod(shape))
        d, psf, _ = gaussian_nuclei_volume(rng, shape, (sxy, sxy, sz),
                                           int(round(40 * n / 131072)),
                                           int(round(20 * n / 131072)), background=10.0)
        out.append(dict(shape=shape, sigma=(sxy, sxy, sz), d=d, psf=psf, u0=initial_estimate(d)))
    return out
