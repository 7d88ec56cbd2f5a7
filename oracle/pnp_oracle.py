"""Plug-and-play ADMM deblurring around the G-BM3D denoiser: the workload
that motivates fast repeated denoising (many denoiser calls per restored
image, Sec. 1).

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests do.  It shares no code with the GPU
library or its driver.

The loop is the textbook plug-and-play ADMM for y = k (*) x + n (periodic
blur, white noise of deviation sigma_n) with a denoiser D_s in place of the
prior's proximal step:

    x <- argmin_x |k (*) x - y|^2 + mu |x - (v - u)|^2      (closed form in
         the Fourier domain, mu = (sigma_n / s)^2)
    v <- D_s(Q(x + u))                                       (Q: uint16
         quantisation of the denoiser input, D_s: two-stage G-BM3D at s)
    u <- u + x - v

with the denoiser strength s decreasing geometrically from s0 to s1 over
the iterations.
"""
from __future__ import annotations

import numpy as np

from . import gbm3d_oracle as O


def x_step(Y: np.ndarray, Kf: np.ndarray, w: np.ndarray, mu: float) -> np.ndarray:
    """argmin_x |k (*) x - y|^2 + mu |x - w|^2 with Y = F(y), Kf = F(k)."""
    X = (np.conj(Kf) * Y + mu * np.fft.fft2(w)) / (np.abs(Kf) ** 2 + mu)
    return np.real(np.fft.ifft2(X))


def strengths(iters: int, s0: float, s1: float) -> np.ndarray:
    """Geometric schedule of denoiser strengths from s0 down to s1."""
    if iters == 1:
        return np.array([s0])
    return s0 * (s1 / s0) ** (np.arange(iters) / (iters - 1))


def gbm3d_denoiser(params: O.Params = O.DEFAULT):
    """D_s(q): two-stage G-BM3D of the uint16 image q at strength s."""
    return lambda q, s: O.denoise(q, float(s), params)[0]


def pnp_admm(y: np.ndarray, Kf: np.ndarray, sigma_n: float, iters: int, s0: float, s1: float,
             params: O.Params = O.DEFAULT, denoiser=None):
    """Restored image x and the last denoiser output v after `iters` rounds.
    denoiser(q, s) maps the uint16 image q and the strength s to the prior
    step's output (default: the two-stage G-BM3D with `params`)."""
    D = gbm3d_denoiser(params) if denoiser is None else denoiser
    Y = np.fft.fft2(y)
    x = y.copy()
    v = y.copy()
    u = np.zeros_like(y)
    for s in strengths(iters, s0, s1):
        mu = (sigma_n / s) ** 2
        x = x_step(Y, Kf, v - u, mu)
        v = D(O.quantize(x + u), s)
        u = u + x - v
    return x, v
