"""Plug-and-play ADMM deblurring with the library's denoiser (a workload
driver: the motivating use of fast repeated denoising, Sec. 1).

For observations y = k (*) x + n (periodic blur, white noise of deviation
sigma_n) each round runs

    x <- argmin_x |k (*) x - y|^2 + mu |x - (v - u)|^2   (Fourier closed form,
         mu = (sigma_n / s)^2; torch FFTs)
    v <- G-BM3D_s(Q(x + u))                              (gbm3d_quantize, then
         one gbm3d_denoise_batch call for all images, replayed as a graph)
    u <- u + x - v

with the denoiser strength s going geometrically from s0 to s1.  Every
denoising step runs in the library's kernels; the data step and the dual
update are plain tensor arithmetic around them.
"""
from __future__ import annotations

import numpy as np

from . import synth


def strengths(iters: int, s0: float, s1: float) -> np.ndarray:
    if iters == 1:
        return np.array([s0])
    return s0 * (s1 / s0) ** (np.arange(iters) / (iters - 1))


def run(ctx, y, psf: np.ndarray, sigma_n: float, iters: int = 30, s0: float = 20 / 255, s1: float = 4 / 255,
        graph: bool = True, params=None, events: bool = False):
    """Restore a batch y (float32 CUDA tensor [B, H, W]); returns (x, v) and,
    with events, the time spent in the denoiser calls and in total (ms)."""
    import torch
    B, H, W = y.shape
    dev = y.device
    Kf = torch.from_numpy(synth.psf_spectrum(psf, H, W)[:, : W // 2 + 1]).to(dev, torch.complex64)
    Yf = torch.fft.rfft2(y)
    KtY = torch.conj(Kf) * Yf
    K2 = (Kf.real ** 2 + Kf.imag ** 2)
    x = y.clone()
    v = y.clone()
    u = torch.zeros_like(y)
    zq = torch.empty((B, H, W), dtype=torch.uint16, device=dev)
    outs = [v[b] for b in range(B)]
    ins = [zq[b] for b in range(B)]
    marks = []
    if events:
        t0, t1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        t0.record()
    for s in strengths(iters, s0, s1):
        mu = float((sigma_n / s) ** 2)
        X = (KtY + mu * torch.fft.rfft2(v - u)) / (K2 + mu)
        x = torch.fft.irfft2(X, s=(H, W))
        ctx.quantize((x + u).contiguous(), out=zq)
        if events:
            marks.append((torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)))
            marks[-1][0].record()
        ctx.denoise_batch(ins, [float(s)] * B, outs=outs, params=params, graph=graph)
        if events:
            marks[-1][1].record()
        u += x - v
    if events:
        t1.record()
        torch.cuda.synchronize()
        d_ms = sum(a.elapsed_time(b) for a, b in marks)
        return x, v, {"denoise_ms": d_ms, "total_ms": t0.elapsed_time(t1)}
    return x, v


def bench(ctx, n: int = 8, size: int = 256, iters: int = 30, sigma_n: float = 0.01, seed: int = 7000):
    """Throughput of the loop on n seeded size x size images: rounds per
    second, denoiser Mpixel/s inside the loop, and PSNR before and after."""
    import torch
    from .gbm3d import psnr_db
    cases = [synth.pnp_case(size, size, seed + i, sigma_n) for i in range(n)]
    psf = cases[0][2]
    y = torch.from_numpy(np.stack([c[1] for c in cases]).astype(np.float32)).cuda()
    run(ctx, y, psf, sigma_n, iters=2)                       # warm-up: graph capture
    torch.cuda.synchronize()
    x, v, t = run(ctx, y, psf, sigma_n, iters=iters, events=True)
    xs = x.cpu().numpy()
    p_in = float(np.mean([psnr_db(c[1], c[0]) for c in cases]))
    p_out = float(np.mean([psnr_db(xs[i], cases[i][0]) for i in range(n)]))
    mpx = n * size * size / 1e6
    return {"images": n, "size": size, "iterations": iters, "sigma_n_255": sigma_n * 255,
            "ms_per_round": t["total_ms"] / iters, "denoise_ms_per_round": t["denoise_ms"] / iters,
            "denoise_mpix_s": mpx * iters / (t["denoise_ms"] * 1e-3),
            "psnr_observed_db": p_in, "psnr_restored_db": p_out}
