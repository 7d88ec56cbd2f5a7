"""Global stage 1 of G-BM3D (the hard-threshold estimate as one volume):
plain float64 CPU oracle.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests do.  It shares no code with the GPU
library.

What it computes (Sec. 3, "global" filtering; Sec. 5 parameter list):

* reference blocks z_N^{pq} of side N tile the image: top-left (pN, qN);
* each is matched to its K nearest blocks in the search window (Sec. 3.1,
  S^K_pq; same exact distance, key and tie rule as the grouped path, the
  reference itself in slot 0);
* the volume V[pN + a, qN + b, k] = z^{ij_k}[a, b] stacks the k-th match of
  every reference behind the reference's own tile (slot 0 is the noisy
  image itself);
* U_h = S_{-h} T^{-1}(Upsilon(T(S_h V))) for the cycle spins h = 0 .. H-1,
  S_h a circular shift by h in each of the three dimensions, averaged;
* every filtered block is added back at its source position with weight
  w_pq = 1 / TV(u^{pq}) (3-D total variation of the reference's N x N x K
  block of U) and normalised;
* the whole procedure phi is repeated on translated images and averaged:
  Y_f = mean_h S_{-h} phi(S_h Z) (eq. firstEst).

Readings of points the paper leaves open (listed with their reasons in the
design notes):

* T is the separable periodic 3-D Mallat decomposition with three levels:
  each level applies the one-level bior1.5 analysis step along both spatial
  axes and the orthonormal one-level Haar step along the match axis to the
  current low-low-low sub-volume;
* a coefficient in a detail band of level l (1 finest .. 3 coarsest) is hard
  thresholded at tau_l = sigma (3.6 - 0.3 l); the final approximation is
  kept;
* TV is the anisotropic L1 norm of forward differences along the three
  axes of u^{pq} (not periodic), w = 1 / (TV + eps), eps = tv_eps_rel *
  sigma * N^2 * K;
* the translations are h = 0 and N/4 along both axes (two repeated trials,
  Sec. 5; eq. firstEst lists N/2 as a third), the cycle spins h = 0, 1;
* image sides that are not multiples of N are mirror-padded (mirror_pad), as
  the paper does, and the estimate is cropped back.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

from . import gbm3d_oracle as O


@dataclass(frozen=True)
class GlobalParams:
    patch: int = 16            # N (Sec. 5: block size of the first step)
    search: int = 33           # odd search window side (Sec. 5 states 32)
    k: int = 16                # matched blocks per reference (Sec. 3)
    levels: int = 3            # wavelet levels (Sec. 5)
    cycles: int = 2            # cycle spins h = 0 .. cycles-1 (Sec. 3, Sec. 5)
    shifts: tuple = (0, 4)     # image translations (eq. firstEst, Sec. 5 trials)
    ht_a: float = 3.6
    ht_b: float = 0.3
    tv_eps_rel: float = 1e-3

    def with_(self, **kw) -> "GlobalParams":
        return replace(self, **kw)


GDEFAULT = GlobalParams()


def tile_refs(H: int, W: int, N: int):
    """Top-left corners of the reference tiles, raster order."""
    ry = np.repeat(np.arange(0, H, N), W // N)
    rx = np.tile(np.arange(0, W, N), H // N)
    return ry, rx


def match_tiles(Z: np.ndarray, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """Displacement ranks [n_tiles, K] of every reference tile's matches."""
    H, W = Z.shape
    ry, rx = tile_refs(H, W, p.patch)
    return O.select_matches(O.block_distances(Z, ry, rx, p.patch, p.search), p.k, p.search)


def build_volume(z: np.ndarray, idx: np.ndarray, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """V[k, y, x] (match axis first): slot k of the tile holding (y, x)."""
    H, W = z.shape
    N, K = p.patch, p.k
    ry, rx = tile_refs(H, W, N)
    py, px = O.match_positions(H, W, idx, ry, rx, p.search)          # [G, K]
    blocks = O._blocks(z, py.ravel(), px.ravel(), N).reshape(len(ry), K, N, N)
    V = np.empty((K, H, W))
    for g in range(len(ry)):
        V[:, ry[g]:ry[g] + N, rx[g]:rx[g] + N] = blocks[g]
    return V


def _haar_step(L: int) -> np.ndarray:
    """One orthonormal Haar level on length L: sums (x0 + x1)/sqrt2 first,
    differences (x0 - x1)/sqrt2 second."""
    A = np.zeros((L, L))
    for n in range(L // 2):
        A[n, 2 * n] = A[n, 2 * n + 1] = 1.0 / np.sqrt(2.0)
        A[L // 2 + n, 2 * n] = 1.0 / np.sqrt(2.0)
        A[L // 2 + n, 2 * n + 1] = -1.0 / np.sqrt(2.0)
    return A


def _apply(M: np.ndarray, X: np.ndarray, axis: int) -> np.ndarray:
    return np.moveaxis(np.tensordot(M, X, axes=([1], [axis])), 0, axis)


def dwt3(V: np.ndarray, levels: int) -> np.ndarray:
    """Separable periodic 3-D Mallat decomposition of V[k, y, x]."""
    C = np.array(V, dtype=np.float64, copy=True)
    K, H, W = C.shape
    for j in range(levels):
        k, h, w = K >> j, H >> j, W >> j
        sub = C[:k, :h, :w]
        sub = _apply(O.bior15_analysis_matrix(h), sub, 1)
        sub = _apply(O.bior15_analysis_matrix(w), sub, 2)
        sub = _apply(_haar_step(k), sub, 0)
        C[:k, :h, :w] = sub
    return C


def idwt3(C: np.ndarray, levels: int) -> np.ndarray:
    V = np.array(C, dtype=np.float64, copy=True)
    K, H, W = V.shape
    for j in reversed(range(levels)):
        k, h, w = K >> j, H >> j, W >> j
        sub = V[:k, :h, :w]
        sub = _apply(_haar_step(k).T, sub, 0)
        sub = _apply(np.linalg.inv(O.bior15_analysis_matrix(w)), sub, 2)
        sub = _apply(np.linalg.inv(O.bior15_analysis_matrix(h)), sub, 1)
        V[:k, :h, :w] = sub
    return V


def coefficient_levels(K: int, H: int, W: int, levels: int) -> np.ndarray:
    """Level of each 3-D coefficient: l >= 1 for detail bands (1 finest),
    0 for the final approximation."""
    kk, yy, xx = np.meshgrid(np.arange(K), np.arange(H), np.arange(W), indexing="ij")
    lev = np.zeros((K, H, W), dtype=np.int64)
    for j in range(1, levels + 1):        # nested regions: the coarser level overwrites
        inside = (kk < (K >> (j - 1))) & (yy < (H >> (j - 1))) & (xx < (W >> (j - 1)))
        lev[inside] = j
    approx = (kk < (K >> levels)) & (yy < (H >> levels)) & (xx < (W >> levels))
    lev[approx] = 0
    return lev


def filter_volume(V: np.ndarray, sigma: float, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """U = mean over cycle spins h of S_{-h} T^{-1} Upsilon T S_h V."""
    K, H, W = V.shape
    lev = coefficient_levels(K, H, W, p.levels)
    tau = np.where(lev > 0, sigma * (p.ht_a - p.ht_b * lev), 0.0)
    U = np.zeros_like(V)
    for h in range(p.cycles):
        C = dwt3(np.roll(V, (h, h, h), axis=(0, 1, 2)), p.levels)
        C = O.hard_threshold(C, tau)
        U += np.roll(idwt3(C, p.levels), (-h, -h, -h), axis=(0, 1, 2))
    return U / p.cycles


def tv_weights(U: np.ndarray, sigma: float, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """w_pq = 1 / (TV(u^{pq}) + eps) for every tile, raster order."""
    K, H, W = U.shape
    N = p.patch
    ry, rx = tile_refs(H, W, N)
    w = np.empty(len(ry))
    eps = p.tv_eps_rel * sigma * N * N * K
    for g in range(len(ry)):
        u = U[:, ry[g]:ry[g] + N, rx[g]:rx[g] + N]
        tv = np.abs(np.diff(u, axis=0)).sum() + np.abs(np.diff(u, axis=1)).sum() + np.abs(np.diff(u, axis=2)).sum()
        w[g] = 1.0 / (tv + eps)
    return w


def phi(Z: np.ndarray, sigma: float, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """One pass: match the tiles, filter the volume, aggregate, normalise."""
    H, W = Z.shape
    if H % p.patch or W % p.patch:
        raise ValueError("image sides must be multiples of the block size")
    z = Z.astype(np.float64) / O.U16_MAX
    idx = match_tiles(Z, p)
    U = filter_volume(build_volume(z, idx, p), sigma, p)
    w = tv_weights(U, sigma, p)
    N, K = p.patch, p.k
    ry, rx = tile_refs(H, W, N)
    py, px = O.match_positions(H, W, idx, ry, rx, p.search)
    blocks = np.stack([U[:, ry[g]:ry[g] + N, rx[g]:rx[g] + N] for g in range(len(ry))])  # [G, K, N, N]
    num, den = O.aggregate(H, W, blocks, w, py, px)
    return num / den


def mirror_pad(Z: np.ndarray, N: int) -> np.ndarray:
    """Z extended past its bottom and right edges with mirrored values up to
    the next multiples of N (Sec. 3.1: sizes that are not multiples of the
    block size are padded with mirrored image values).  Reading: the edge
    pixel is repeated first, row (column) L + i takes row L - 1 - i, and only
    the ends are padded."""
    H, W = Z.shape
    return np.pad(Z, ((0, (-H) % N), (0, (-W) % N)), mode="symmetric")


def global_basic(Z: np.ndarray, sigma: float, p: GlobalParams = GDEFAULT) -> np.ndarray:
    """Y_f = mean over translations h of S_{-h} phi(S_h Z); an image whose
    sides are not multiples of N is filtered mirror-padded and cropped."""
    H, W = Z.shape
    if H % p.patch or W % p.patch:
        return global_basic(mirror_pad(Z, p.patch), sigma, p)[:H, :W]
    Y = np.zeros(Z.shape)
    for h in p.shifts:
        Y += np.roll(phi(np.roll(Z, (h, h), axis=(0, 1)), sigma, p), (-h, -h), axis=(0, 1))
    return Y / len(p.shifts)
