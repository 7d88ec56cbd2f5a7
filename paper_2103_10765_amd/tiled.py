"""Large images as overlapping sub-images (Sec. 5): the image is cut into
sub-images of side 256 + N (N = 8, the block side) starting every 256
pixels, each is denoised as an image of its own, and the estimate is
stitched back after each stage.

Both stages of all sub-images go through the library's batched call
(gbm3d_denoise_batch: stage 1 only, then stage 2 with each sub-image's piece
of the stitched, quantised pilot).  Stitching gives every pixel the value of
one sub-image: consecutive sub-images split their overlap at its middle.
Here the stitching and the cutting of sub-images are device-to-device
copies of strided slices; all filtering runs in the library.
"""
from __future__ import annotations

import torch

from . import gbm3d

SIZE = 256 + 8
STRIDE = 256


def sub_ranges(n: int, size: int = SIZE, stride: int = STRIDE):
    """Per sub-image along one axis of length n: (start, side, first, end),
    the sub-image covering [start, start + side) and supplying [first, end)."""
    if size >= n:
        return [(0, n, 0, n)]
    first_starts = list(range(0, n - size, stride))
    starts = first_starts + ([n - size] if not first_starts or first_starts[-1] != n - size else [])
    out = []
    for k, a in enumerate(starts):
        left = 0 if k == 0 else (starts[k - 1] + size + a) // 2
        right = n if k + 1 == len(starts) else (a + size + starts[k + 1]) // 2
        out.append((a, size, left, right))
    return out


def _pieces(H: int, W: int, size: int, stride: int):
    return [(ry, rx) for ry in sub_ranges(H, size, stride) for rx in sub_ranges(W, size, stride)]


def _cut(img: torch.Tensor, pieces):
    return [img[y0:y0 + h, x0:x0 + w].contiguous() for (y0, h, _, _), (x0, w, _, _) in pieces]


def _stitch(parts, pieces, out: torch.Tensor):
    for P, ((y0, _, ya, yb), (x0, _, xa, xb)) in zip(parts, pieces):
        out[ya:yb, xa:xb].copy_(P[ya - y0:yb - y0, xa - x0:xb - x0])
    return out


def denoise(ctx: gbm3d.Context, noisy: torch.Tensor, sigma: float, size: int = SIZE, stride: int = STRIDE,
            params: gbm3d.Params | None = None, out: torch.Tensor | None = None):
    """Two-stage G-BM3D of a uint16 CUDA image on sub-images.  Returns
    (out float32 [H, W], basic float32 [H, W], pilot uint16 [H, W])."""
    H, W = (int(v) for v in noisy.shape)
    pieces = _pieces(H, W, size, stride)
    subs = _cut(noisy, pieces)
    sig = [sigma] * len(subs)
    basic = _stitch(ctx.denoise_batch(subs, sig, params=params, basic_only=True), pieces,
                    torch.empty((H, W), dtype=torch.float32, device=noisy.device))
    pilot = ctx.quantize(basic)
    if out is None:
        out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
    _stitch(ctx.denoise_batch(subs, sig, pilots=_cut(pilot, pieces), params=params), pieces, out)
    return out, basic, pilot
