"""Pins of the plug-and-play deblurring oracle (CPU only)."""
import numpy as np

from oracle import pnp_oracle as P
from paper_2103_10765_amd import synth


def _conv_periodic(x, k):
    """k (*) x by explicit periodic shifts, the PSF centred at (0, 0)."""
    s = k.shape[0]
    c = s // 2
    out = np.zeros_like(x)
    for a in range(s):
        for b in range(s):
            out += k[a, b] * np.roll(x, (a - c, b - c), axis=(0, 1))
    return out


def test_psf_spectrum_is_the_periodic_convolution():
    rng = np.random.default_rng(0)
    x = rng.random((20, 23))
    k = synth.blur_kernel(9, 1.6)
    via_fft = np.real(np.fft.ifft2(np.fft.fft2(x) * synth.psf_spectrum(k, 20, 23)))
    assert np.abs(via_fft - _conv_periodic(x, k)).max() < 1e-12


def test_x_step_solves_the_normal_equations():
    """(K'K + mu I) x = K'y + mu w, with K the periodic blur and K' its
    adjoint (the flipped PSF; the Gaussian is symmetric)."""
    rng = np.random.default_rng(1)
    H, W = 24, 30
    k = synth.blur_kernel(9, 1.6)
    y, w = rng.random((H, W)), rng.random((H, W))
    mu = 0.37
    x = P.x_step(np.fft.fft2(y), synth.psf_spectrum(k, H, W), w, mu)
    kf = k[::-1, ::-1]
    lhs = _conv_periodic(_conv_periodic(x, k), kf) + mu * x
    rhs = _conv_periodic(y, kf) + mu * w
    assert np.abs(lhs - rhs).max() < 1e-10


def test_x_step_without_blur_is_the_weighted_mean():
    rng = np.random.default_rng(2)
    y, w = rng.random((16, 16)), rng.random((16, 16))
    delta = np.zeros((3, 3))
    delta[1, 1] = 1.0
    x = P.x_step(np.fft.fft2(y), synth.psf_spectrum(delta, 16, 16), w, 0.25)
    assert np.abs(x - (y + 0.25 * w) / 1.25).max() < 1e-12


def test_strength_schedule():
    s = P.strengths(5, 0.08, 0.02)
    assert abs(s[0] - 0.08) < 1e-15 and abs(s[-1] - 0.02) < 1e-15
    assert np.allclose(s[1:] / s[:-1], (0.02 / 0.08) ** 0.25)


def test_observation_model():
    clean, y, k = synth.pnp_case(96, 96, 3, sigma_n=0.02)
    assert abs(k.sum() - 1.0) < 1e-12 and np.allclose(k, k.T)
    resid = y - np.real(np.fft.ifft2(np.fft.fft2(clean) * synth.psf_spectrum(k, 96, 96)))
    assert abs(resid.std() - 0.02) < 0.002


def test_admm_rounds_by_hand():
    """Three rounds of the loop on a constant image with no blur and an affine
    stand-in denoiser D(q, s) = q / 65535 / 2 + s, derived by hand from the
    textbook plug-and-play ADMM: x = (y + mu (v - u)) / (1 + mu) with
    mu = (sigma_n / s)^2 (the x-step without blur), v = D(Q(x + u)), and the
    dual update u <- u + x - v; strengths geometric from s0 to s1."""
    H, W = 6, 5
    c, sn, s0, s1 = 0.4, 0.03, 0.08, 0.02
    y = np.full((H, W), c)
    delta = np.zeros((3, 3))
    delta[1, 1] = 1.0
    Kf = synth.psf_spectrum(delta, H, W)

    def D(q, s):
        return q.astype(np.float64) / 65535.0 / 2.0 + s

    def Q(t):
        return np.floor(min(max(t, 0.0), 1.0) * 65535.0 + 0.5) / 65535.0

    x, v, u = c, c, 0.0
    for s in (s0, s0 * (s1 / s0) ** 0.5, s1):
        mu = (sn / s) ** 2
        x = (c + mu * (v - u)) / (1.0 + mu)
        v = Q(x + u) / 2.0 + s
        u = u + x - v
    gx, gv = P.pnp_admm(y, Kf, sn, 3, s0, s1, denoiser=D)
    assert np.abs(gx - x).max() < 1e-12 and np.abs(gv - v).max() < 1e-12
    # the hand derivation is not degenerate: the dual variable and the
    # strength schedule both change the result
    assert abs(x - c) > 1e-3 and abs(u) > 1e-3
