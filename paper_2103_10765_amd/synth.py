"""Seeded synthetic test images for the G-BM3D hot path.

This module only draws inputs: piecewise-smooth shapes with sinusoidal
texture on a tilted plane, additive Gaussian noise of a given standard
deviation, and uint16 quantisation of the noisy image.  It holds none of the
denoiser's arithmetic, so both the GPU path and the CPU oracle can be fed from
it without sharing any of the method.

The paper evaluates on eight natural photographs (Sec. 5, Table 1) that are
not available here; these images stand in for them.  Noise follows the
paper's model of i.i.d. zero-mean Gaussian noise of standard deviation sigma
(Sec. 5), with sigma on the [0, 1] intensity scale.
"""
from __future__ import annotations

import numpy as np

U16_MAX = 65535.0


def _paint(img: np.ndarray, rng: np.random.Generator, n_shapes: int) -> None:
    H, W = img.shape
    m = min(H, W)
    for _ in range(n_shapes):
        kind = int(rng.integers(0, 3))          # 0 ellipse, 1 rectangle, 2 half-plane triangle
        size = rng.uniform(0.05, 0.3) * m
        cy, cx = rng.uniform(0, H), rng.uniform(0, W)
        ar = rng.uniform(0.5, 2.0)
        ry, rx = size * np.sqrt(ar) / 2, size / np.sqrt(ar) / 2
        theta = rng.uniform(0, np.pi)
        c0 = rng.uniform(0, 1)
        ramp = rng.uniform(-0.5, 0.5) / max(size, 1.0) if rng.uniform() < 0.5 else 0.0
        ramp_dir = rng.uniform(0, 2 * np.pi)
        tex = rng.uniform() < 0.5
        amp = rng.uniform(0.03, 0.12)
        freq = rng.uniform(1 / 32, 1 / 4)
        fdir = rng.uniform(0, 2 * np.pi)
        phase = rng.uniform(0, 2 * np.pi)
        rad = int(np.ceil(max(ry, rx) * 1.5)) + 1
        y0, y1 = max(0, int(cy) - rad), min(H, int(cy) + rad + 1)
        x0, x1 = max(0, int(cx) - rad), min(W, int(cx) + rad + 1)
        if y0 >= y1 or x0 >= x1:
            continue
        yy, xx = np.mgrid[y0:y1, x0:x1].astype(np.float64)
        dy, dx = yy - cy, xx - cx
        u = dx * np.cos(theta) + dy * np.sin(theta)
        v = -dx * np.sin(theta) + dy * np.cos(theta)
        if kind == 0:
            mask = (u / rx) ** 2 + (v / ry) ** 2 <= 1.0
        elif kind == 1:
            mask = (np.abs(u) <= rx) & (np.abs(v) <= ry)
        else:
            # a triangle: intersection of three half-planes around the centre
            mask = np.ones_like(u, dtype=bool)
            for j in range(3):
                a = theta + 2 * np.pi * j / 3
                mask &= (dx * np.cos(a) + dy * np.sin(a)) <= 0.5 * size
        # fill values, evaluated only where the shape covers the image
        mdx, mdy, mxx, myy = dx[mask], dy[mask], xx[mask], yy[mask]
        val = c0 + ramp * (mdx * np.cos(ramp_dir) + mdy * np.sin(ramp_dir))
        if tex:
            val = val + amp * np.sin(2 * np.pi * freq * (mxx * np.cos(fdir) + myy * np.sin(fdir)) + phase)
        sub = img[y0:y1, x0:x1]
        sub[mask] = val


def clean_image(H: int, W: int, seed: int, edge_rects: int = 0) -> np.ndarray:
    """Piecewise-smooth float64 image in [0, 1] of shape (H, W)."""
    rng = np.random.default_rng(seed)
    b0 = rng.uniform(0.2, 0.8)
    gx, gy = rng.uniform(-0.2, 0.2, size=2)
    yy = np.arange(H, dtype=np.float64)[:, None] / H
    xx = np.arange(W, dtype=np.float64)[None, :] / W
    img = b0 + gx * xx + gy * yy
    img = np.broadcast_to(img, (H, W)).copy()
    n_shapes = min(64, 8 + (H * W) // 16384)
    _paint(img, rng, n_shapes)
    for _ in range(edge_rects):
        h, w = rng.integers(4, 65, size=2)
        y, x = rng.integers(0, H), rng.integers(0, W)
        img[y:y + h, x:x + w] = rng.uniform(0, 1)
    return np.clip(img, 0.0, 1.0)


def add_noise(clean: np.ndarray, sigma: float, seed: int) -> np.ndarray:
    """Noisy uint16 image: clip(clean + N(0, sigma^2), 0, 1) quantised to 16 bits."""
    rng = np.random.default_rng(seed + 1_000_000)
    noisy = np.clip(clean + sigma * rng.standard_normal(clean.shape), 0.0, 1.0)
    return np.floor(noisy * U16_MAX + 0.5).astype(np.uint16)


def make_case(H: int, W: int, sigma: float, seed: int, edge_rects: int = 0):
    """(clean float64 image, noisy uint16 image) for one seeded case."""
    clean = clean_image(H, W, seed, edge_rects)
    return clean, add_noise(clean, sigma, seed)


def to_u16(x: np.ndarray) -> np.ndarray:
    """Quantise a [0, 1] float image to uint16 (used to make pilot inputs)."""
    return np.floor(np.clip(x, 0.0, 1.0) * U16_MAX + 0.5).astype(np.uint16)


# ---- the workload recipes --------------------------------------------------

SIGMA25 = 25.0 / 255.0


def single_image_case(size: int = 512, sigma: float = SIGMA25, seed: int = 2):
    return make_case(size, size, sigma, seed)


def large_image_case(size: int = 4096, sigma: float = SIGMA25, seed: int = 4):
    return make_case(size, size, sigma, seed, edge_rects=600)


def batch_specs(n: int = 64, lo: int = 256, hi: int = 1024, seed: int = 3000):
    """Per-image (H, W, sigma, seed) for a batch of uneven sizes."""
    rng = np.random.default_rng(seed)
    H = rng.integers(lo, hi + 1, size=n)
    W = rng.integers(lo, hi + 1, size=n)
    sig = rng.uniform(10.0, 50.0, size=n) / 255.0
    return [(int(H[i]), int(W[i]), float(sig[i]), seed + 1 + i) for i in range(n)]


def batch_cases(specs):
    return [make_case(h, w, s, sd) for (h, w, s, sd) in specs]


def pilot_train_sigmas(n: int = 20000, seed: int = 5000):
    rng = np.random.default_rng(seed)
    return rng.uniform(10.0, 50.0, size=n) / 255.0


def pilot_train_crop(i: int, sigma: float, size: int = 128):
    return make_case(size, size, sigma, 500_000 + i)


def pilot_eval_cases(n: int = 32, size: int = 512, sigma: float = SIGMA25):
    return [make_case(size, size, sigma, 6000 + i) for i in range(n)]


# ---- plug-and-play deblurring workload -------------------------------------

def blur_kernel(size: int = 9, std: float = 1.6) -> np.ndarray:
    """Normalised isotropic Gaussian point-spread function (size x size)."""
    a = np.arange(size, dtype=np.float64) - (size - 1) / 2.0
    g = np.exp(-0.5 * (a / std) ** 2)
    k = np.outer(g, g)
    return k / k.sum()


def psf_spectrum(k: np.ndarray, H: int, W: int) -> np.ndarray:
    """2-D DFT (H x W) of the point-spread function centred at pixel (0, 0),
    so that multiplying spectra is a zero-phase periodic convolution."""
    s = k.shape[0]
    pad = np.zeros((H, W))
    pad[:s, :s] = k
    pad = np.roll(pad, (-(s // 2), -(s // 2)), axis=(0, 1))
    return np.fft.fft2(pad)


def pnp_case(H: int, W: int, seed: int, sigma_n: float = 0.01, ksize: int = 9, kstd: float = 1.6):
    """(clean, observation y = k (*) clean + n as float64, psf k): periodic
    blur by a Gaussian PSF and white Gaussian noise of deviation sigma_n."""
    clean = clean_image(H, W, seed)
    k = blur_kernel(ksize, kstd)
    blurred = np.real(np.fft.ifft2(np.fft.fft2(clean) * psf_spectrum(k, H, W)))
    rng = np.random.default_rng(seed + 2_000_000)
    return clean, blurred + sigma_n * rng.standard_normal((H, W)), k
