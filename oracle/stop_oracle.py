"""FP64 CPU oracle for metric-guided automatic stopping of Richardson-Lucy.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it, and it imports nothing from the GPU package.

The paper (§4.3, "Richardson-Lucy algorithm" and its evaluation paragraph)
monitors an image-quality metric after each iteration and stops once its
improvement between consecutive iterations falls below a configurable
threshold; the metrics it names are PSNR against ground truth (the
scale-invariant form of Weigert et al., 2018) and SSIM, and a resolution
derived from single-image Fourier ring correlation.  It states neither the
threshold's value nor the exact comparison.  Readings (listed with their
reasons in the design notes):

* "loglik": the Poisson log-likelihood l_k = sum_{q>eps} (d log q - q) of the
  estimate u_k entering iteration k (q = H u_k), the objective RL maximises;
  improvement (l_k - l_{k-1}) / |l_k|; when it drops below the threshold at
  iteration k >= 1 that iteration is not carried out and u_k is returned.
* "change": m_k = ||u_{k+1} - u_k|| / ||u_k|| after iteration k; stop once
  m_k < threshold, returning u_{k+1}.
* "psnr": scale-invariant PSNR of u_{k+1} against a reference volume g,
  20 log10(max g - min g) - 10 log10(MSE of the least-squares affine fit
  a u + b to g); improvement psnr_k - psnr_{k-1} (dB, none at k = 0); stop once it
  is below the threshold, returning u_{k+1}.
* "fsc": the single-image FSC resolution of u_{k+1} (``fsc_oracle``: FSC of the
  two diagonal half-size sub-volumes, frequency where it first drops below
  `fsc_threshold`, default 1/7); improvement r_k - r_{k-1} (cycles per voxel,
  none at k = 0); stop once it is below the threshold, returning u_{k+1}.
* "ssim": mean SSIM of u_{k+1} against the reference (``ssim_oracle``);
  improvement ssim_k - ssim_{k-1} (none at k = 0); stop once it is below the
  threshold, returning u_{k+1}.
* No stop before `min_iter` iterations have been carried out; at most
  `max_iter` iterations.
"""

from __future__ import annotations

import numpy as np

from . import fsc_oracle, ssim_oracle
from .rl_oracle import EPS, adjoint, forward, loglik, otf, ratio

METRICS = ("loglik", "change", "psnr", "fsc", "ssim")


def fsc_resolution(u, nbins: int = 64, fsc_threshold: float = 1.0 / 7.0) -> float:
    """Single-image FSC resolution (cycles per voxel) of u."""
    a, b = fsc_oracle.split_diagonal(u)
    return fsc_oracle.resolution(fsc_oracle.fsc(a, b, nbins), nbins, fsc_threshold)


def psnr_si(u, g) -> float:
    """Scale-invariant PSNR (dB) of u against g: affine least-squares fit of u to g,
    then 20 log10(range of g) - 10 log10(mean squared residual)."""
    u = np.asarray(u, dtype=np.float64).ravel()
    g = np.asarray(g, dtype=np.float64).ravel()
    du, dg = u - u.mean(), g - g.mean()
    cuu, cug, cgg = float(du @ du), float(du @ dg), float(dg @ dg)
    sse = cgg - (cug * cug / cuu if cuu > 0 else 0.0)
    mse = max(sse, 0.0) / u.size
    rng = float(g.max() - g.min())
    return 20.0 * np.log10(rng) - 10.0 * np.log10(mse)


def rel_change(u_new, u_old) -> float:
    """||u_new - u_old|| / ||u_old|| in FP64."""
    a = np.asarray(u_new, dtype=np.float64)
    b = np.asarray(u_old, dtype=np.float64)
    return float(np.linalg.norm((a - b).ravel()) / np.linalg.norm(b.ravel()))


def rl_stop(d, h, u0, max_iter: int, metric: str, threshold: float, reference=None,
            min_iter: int = 0, eps: float = EPS, nbins: int = 64,
            fsc_threshold: float = 1.0 / 7.0):
    """Richardson-Lucy with metric-guided stopping.

    Returns (u, n_done, history): the estimate after the iterations carried out,
    their number, and the metric value computed at each check (loglik: l_0 ..
    l_k; change and psnr: m_0 .. m_{n_done-1}).
    """
    if metric not in METRICS:
        raise ValueError(f"metric must be one of {METRICS}")
    if metric in ("psnr", "ssim") and reference is None:
        raise ValueError(f"{metric} needs a reference volume")
    d = np.asarray(d, dtype=np.float64)
    u = np.array(u0, dtype=np.float64, copy=True)
    K = otf(h)
    hist = []
    n_done = 0
    for k in range(max_iter):
        q = forward(u, K)
        if metric == "loglik":
            hist.append(loglik(d, q, eps))
            if k >= 1 and k >= min_iter:
                if (hist[k] - hist[k - 1]) / abs(hist[k]) < threshold:
                    break
        u_new = u * np.maximum(adjoint(ratio(d, q, eps), K), 0.0)
        n_done = k + 1
        stop = False
        if metric == "change":
            hist.append(rel_change(u_new, u))
            stop = hist[-1] < threshold
        elif metric == "psnr":
            hist.append(psnr_si(u_new, reference))
            stop = k >= 1 and hist[k] - hist[k - 1] < threshold
        elif metric == "ssim":
            hist.append(ssim_oracle.ssim(u_new, reference))
            stop = k >= 1 and hist[k] - hist[k - 1] < threshold
        elif metric == "fsc":
            hist.append(fsc_resolution(u_new, nbins, fsc_threshold))
            stop = k >= 1 and hist[k] - hist[k - 1] < threshold
        u = u_new
        if stop and n_done >= min_iter:
            break
    return u, n_done, np.array(hist)
