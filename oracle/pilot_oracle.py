"""Plain float64 CPU oracle of the learned pilot network.

TEST INFRASTRUCTURE ONLY: used by the tests, not by the product path.  Shares
no code with the GPU library.

The paper has no learned component; the pilot is an addition that stands in
for stage 1 as the estimate that drives the Wiener stage (Sec. 4 needs only
"the first estimate").  The network: six 3x3 convolutions with zero "same"
padding, channels 2 -> 32 -> 32 -> 32 -> 32 -> 32 -> 1, ReLU after the first
five, input (z, constant sigma plane), residual output pilot = z - f(z, sigma).
Weights and the activations between layers are bfloat16 (round to nearest
even) in the GPU path; `forward(..., bf16=True)` rounds at the same places.

Parameter vector layout (float32 master copy, 37 889 entries): for each layer
in order, the weights W[ky][kx][ci][co] (row-major) followed by the bias[co].
"""
from __future__ import annotations

import numpy as np

LAYERS = [(2, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]


def n_params() -> int:
    return sum(9 * ci * co + co for ci, co in LAYERS)


def unpack(theta: np.ndarray):
    """[(W [3,3,ci,co], b [co]), ...] views of the flat parameter vector."""
    out, o = [], 0
    for ci, co in LAYERS:
        W = theta[o:o + 9 * ci * co].reshape(3, 3, ci, co)
        o += 9 * ci * co
        b = theta[o:o + co]
        o += co
        out.append((W, b))
    assert o == len(theta)
    return out


def bf16_round(x) -> np.ndarray:
    """Round to bfloat16 (via float32, round to nearest, ties to even)."""
    f = np.asarray(x, dtype=np.float32)
    u = f.view(np.uint32).astype(np.uint64)
    r = ((u + 0x7FFF + ((u >> 16) & 1)) & 0xFFFF0000).astype(np.uint32)
    out = r.view(np.float32).astype(np.float64)
    return np.where(np.isfinite(f), out, f.astype(np.float64))


def conv3x3(x: np.ndarray, W: np.ndarray, b: np.ndarray) -> np.ndarray:
    """y[n, i, j, co] = b[co] + sum_{ky,kx,ci} x[n, i+ky-1, j+kx-1, ci] W[ky,kx,ci,co],
    zero outside the image.  x: [N, H, Wd, ci]."""
    N, H, Wd, _ = x.shape
    xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
    y = np.broadcast_to(b, (N, H, Wd, W.shape[3])).astype(np.float64).copy()
    for ky in range(3):
        for kx in range(3):
            y += np.einsum("nhwi,io->nhwo", xp[:, ky:ky + H, kx:kx + Wd, :], W[ky, kx])
    return y


def network_input(z: np.ndarray, sigma) -> np.ndarray:
    """[N, H, W, 2]: the image and a constant plane holding its sigma."""
    z = np.asarray(z, dtype=np.float64)
    s = np.broadcast_to(np.asarray(sigma, dtype=np.float64).reshape(-1, 1, 1), z.shape)
    return np.stack([z, s], axis=-1)


def forward(theta: np.ndarray, z: np.ndarray, sigma, bf16: bool = True):
    """pilot = z - f(z, sigma) and the list of layer inputs (for backward)."""
    params = unpack(np.asarray(theta, dtype=np.float64))
    x = network_input(z, sigma)
    if bf16:
        x = bf16_round(x)
    acts = [x]
    for l, (W, b) in enumerate(params):
        if bf16:
            W, b = bf16_round(W), b
        y = conv3x3(acts[-1], W, b)
        if l < len(params) - 1:
            y = np.maximum(y, 0.0)
            if bf16:
                y = bf16_round(y)
        acts.append(y)
    f = acts[-1][..., 0]
    return np.asarray(z, dtype=np.float64) - f, acts


def loss_and_grad(theta: np.ndarray, z: np.ndarray, sigma, target: np.ndarray, bf16: bool = True, weight=None):
    """Mean squared error of the pilot against `target` (each image's squared
    errors scaled by weight[b] when given) and its gradient with respect to
    theta (backpropagation through the convolutions; ReLU derivative taken as
    1 where the layer output is positive)."""
    params = unpack(np.asarray(theta, dtype=np.float64))
    pilot, acts = forward(theta, z, sigma, bf16)
    diff = pilot - np.asarray(target, dtype=np.float64)
    n = diff.size
    wb = np.ones(diff.shape[0]) if weight is None else np.asarray(weight, dtype=np.float64)
    wd = wb[:, None, None] * diff
    loss = float(np.sum(wd * diff) / n)
    g = (-2.0 / n * wd)[..., None]              # dL/df, one channel
    grads = []
    for l in range(len(params) - 1, -1, -1):
        W, _ = params[l]
        if bf16:
            W = bf16_round(W)
        x = acts[l]
        N, H, Wd, _ = x.shape
        xp = np.pad(x, ((0, 0), (1, 1), (1, 1), (0, 0)))
        dW = np.empty_like(W)
        for ky in range(3):
            for kx in range(3):
                dW[ky, kx] = np.einsum("nhwi,nhwo->io", xp[:, ky:ky + H, kx:kx + Wd, :], g)
        db = g.sum(axis=(0, 1, 2))
        grads.append((dW, db))
        if l > 0:
            gp = np.pad(g, ((0, 0), (1, 1), (1, 1), (0, 0)))
            gx = np.zeros(x.shape)
            for ky in range(3):
                for kx in range(3):
                    gx += np.einsum("nhwo,io->nhwi", gp[:, 2 - ky:2 - ky + H, 2 - kx:2 - kx + Wd, :], W[ky, kx])
            g = gx * (x > 0)
    flat = []
    for dW, db in reversed(grads):
        flat.append(dW.ravel())
        flat.append(db.ravel())
    return loss, np.concatenate(flat)

