"""FP64 CPU oracle for Richardson-Lucy with Biggs-Andrews acceleration.

TEST INFRASTRUCTURE, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the ``cpu_baseline`` leg of ``bench.py`` may
import it, and it imports nothing from the GPU package.

The paper names this variant as the one behind the CUDA Richardson-Lucy tool it
cites (§2, related work, the pycudadecon plugin and its reference to Biggs and
Andrews, 1997).  The method is the first-order vector extrapolation of Biggs &
Andrews, "Acceleration of iterative image restoration algorithms", Applied
Optics 36(8), 1997: an iteration x <- psi(x) is driven from a predicted point
instead of the last iterate,

    h_k   = x_k - x_{k-1}                        (the last step)
    y_k   = max(x_k + alpha_k h_k, 0)            (prediction, kept non-negative)
    x_k+1 = psi(y_k)                             (one plain iteration from y_k)
    g_k   = x_k+1 - y_k                          (what that iteration changed)
    alpha_k = <g_k-1, g_k-2> / <g_k-2, g_k-2>    (clipped to [0, 1])

with alpha_0 = alpha_1 = 0 (two changes are needed before the first estimate of
the acceleration) and alpha = 0 when <g_k-2, g_k-2> = 0.  For Richardson-Lucy
psi(y) = y * max(H^T (d / H y), 0), the plain iteration of ``rl_oracle``.

Readings taken where the cited method leaves a choice (listed with their
reasons in the design notes): the clip of alpha to [0, 1]; the clamp of the
prediction at zero; every call starts the extrapolation afresh from its
initial estimate (no history carried between calls); the flux recorded after
iteration k is sum(x_k+1).

Pinned by a closed form (on a linear contraction psi the iterates and the
alphas follow powers of the contraction factor), by its reduction to the plain
iteration for n_iter <= 2, and by the Richardson-Lucy invariants that hold for
any non-negative starting point (flux conservation, non-negativity, the
delta-PSF fixed point).
"""

from __future__ import annotations

import numpy as np

from .rl_oracle import EPS, adjoint, forward, otf, ratio


def extrapolate(psi, x0, n_iter: int, clamp: bool = True, trace: list | None = None):
    """Biggs-Andrews first-order extrapolation of the map ``psi`` from x0.

    Returns (x_n, alphas) where alphas[k] is the alpha used to predict y_k,
    k = 0..n_iter-1.  If ``trace`` is a list, (raw prediction, y_k) pairs are
    appended to it.
    """
    if n_iter < 0:
        raise ValueError("n_iter must be >= 0")
    x = np.array(x0, dtype=np.float64, copy=True)
    x_prev = None
    g1 = g2 = None  # g_{k-1}, g_{k-2}
    alphas = []
    for k in range(n_iter):
        alpha = 0.0
        if g2 is not None:
            den = float(np.sum(g2 * g2))
            if den > 0.0:
                alpha = min(max(float(np.sum(g1 * g2)) / den, 0.0), 1.0)
        alphas.append(alpha)
        h = x - x_prev if x_prev is not None else np.zeros_like(x)
        raw = x + alpha * h
        y = np.maximum(raw, 0.0) if clamp else raw
        if trace is not None:
            trace.append((raw, y))
        x_next = psi(y)
        g = x_next - y
        g2, g1 = g1, g
        x_prev, x = x, x_next
    return x, np.array(alphas)


def rl_accel(d, h, u0, n_iter: int, eps: float = EPS):
    """Biggs-Andrews accelerated Richardson-Lucy from u0.

    Returns (u, flux, alphas): the FP64 estimate after n_iter iterations, the
    total flux sum(x_k+1) after each iteration, and the alpha of each iteration.
    """
    d = np.asarray(d, dtype=np.float64)
    K = otf(h)
    flux = []

    def psi(y):
        c = adjoint(ratio(d, forward(y, K), eps), K)
        x = y * np.maximum(c, 0.0)
        flux.append(float(x.sum()))
        return x

    u, alphas = extrapolate(psi, u0, n_iter)
    return u, np.array(flux), alphas
