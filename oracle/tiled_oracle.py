"""Large images as overlapping sub-images (Sec. 5): the image is cut into
sub-images of side 256 + N that overlap, each is denoised as an image of its
own, and the estimate is stitched back together after each of the two
stages.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests do.  It shares no code with the GPU
library or its driver.

Readings (the paper names the side and says the pieces overlap and are
stitched after both stages, nothing more):
  * along each axis the sub-images start every `stride` pixels (256) and
    have side `size` (256 + N, N = 8 the block side), the last one ending
    at the image's end; an axis no longer than `size` is one sub-image;
  * each sub-image is filtered with the same periodic boundary as a whole
    image;
  * stitching gives every pixel the value of exactly one sub-image: two
    consecutive sub-images split their overlap at its middle (the pixel is
    taken from the one whose centre is nearer).
"""
from __future__ import annotations

import numpy as np

from . import gbm3d_oracle as O


def axis_plan(L: int, size: int = 264, stride: int = 256):
    """[(start, side, lo, hi)]: the sub-image [start, start + side) supplies
    the pixels [lo, hi) of the stitched axis."""
    if L <= size:
        return [(0, L, 0, L)]
    starts = []
    s = 0
    while s + size < L:
        starts.append(s)
        s += stride
    starts.append(L - size)
    starts = sorted(set(starts))
    plan = []
    for i, s in enumerate(starts):
        lo = 0 if i == 0 else (starts[i - 1] + size + s) // 2
        hi = L if i == len(starts) - 1 else (s + size + starts[i + 1]) // 2
        plan.append((s, size, lo, hi))
    return plan


def _stitch(stage, H: int, W: int, size: int, stride: int) -> np.ndarray:
    """Runs stage(y0, h, x0, w) -> estimate of that sub-image on every
    sub-image and keeps each one's owned pixels."""
    out = np.empty((H, W), dtype=np.float64)
    for (y0, h, ylo, yhi) in axis_plan(H, size, stride):
        for (x0, w, xlo, xhi) in axis_plan(W, size, stride):
            Y = stage(y0, h, x0, w)
            out[ylo:yhi, xlo:xhi] = Y[ylo - y0:yhi - y0, xlo - x0:xhi - x0]
    return out


def denoise(Z: np.ndarray, sigma: float, size: int = 264, stride: int = 256, params: O.Params = O.DEFAULT):
    """Two-stage G-BM3D on sub-images: stage 1 on every sub-image, stitched
    basic estimate, its quantised pilot, stage 2 on every sub-image with the
    pilot's matching sub-image, stitched.  Returns (out, basic, pilot)."""
    H, W = Z.shape
    basic = _stitch(lambda y0, h, x0, w: O.basic_estimate(Z[y0:y0 + h, x0:x0 + w], sigma, params),
                    H, W, size, stride)
    Q = O.quantize(basic)
    out = _stitch(lambda y0, h, x0, w: O.wiener_estimate(Z[y0:y0 + h, x0:x0 + w], Q[y0:y0 + h, x0:x0 + w], sigma,
                                                         params), H, W, size, stride)
    return out, basic, Q
