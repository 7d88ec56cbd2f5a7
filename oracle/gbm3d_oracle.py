"""Plain, slow, float64 CPU oracle for the G-BM3D hot path.

TEST INFRASTRUCTURE ONLY.  Nothing in the product path may import, call or
execute this module; only the tests, the smoke check and the CPU-baseline leg
of the benchmark do.  It shares no code with the GPU library.

What it computes (Sanders & Larkin, "New Computational Techniques for a
Faster Variation of BM3D Image Denoising"):

* periodic image indexing, blocks z^{ij} (Sec. 1.2, eq. (1) and eq. Fblock);
* block distances ||z^{ij} - z^{kl}||^2 (Sec. 2, eq. dfg), evaluated by
  extracting both blocks and summing squared differences in int64;
* arg_K min selection of matched blocks (Sec. 3.1, definition of S^K_pq);
* stage 1: separable 3-D transform of each group (2-D biorthogonal 1.5
  wavelet over the block, 3 levels, and 1-D Haar along the group axis,
  Sec. 5 parameter list), hard thresholding Upsilon (Sec. 3.1) with the
  level-dependent threshold tau_l = sigma (3.6 - 0.3 l) (Sec. 5), inverse,
  1 / TV weights (Sec. 3.1) and the weighted-average aggregation (Sec. 3.1);
* stage 2: 2-D DCT x 1-D Haar empirical Wiener filter driven by the first
  estimate, with block matching on that estimate (Sec. 4, and the two-stage
  description in Sec. 1.1).

Readings of points the paper leaves open (each is listed with its reason in
the design notes):

* references sit on a periodic step-3 grid rather than tiling the image, so
  the cycle spins and translations of Sec. 3 are not applied;
* the search window is every displacement with |dy|, |dx| <= search // 2;
* ties in arg_K are broken by the lower displacement rank
  r = (dy + R) * S + (dx + R); the reference itself is always slot 0;
* the 2-D wavelet is the periodic Mallat decomposition (recursing on the
  low-low band), a 2-D coefficient (u, v) belongs to level
  l = log2(N) - floor(log2(max(u, v))) and the approximation to the coarsest
  level; the 1-D Haar is orthonormal and runs to full depth;
* the 3-D DC coefficient is never shrunk; |alpha| >= lambda keeps;
* TV is the anisotropic L1 norm of forward differences along both block axes
  and the group axis (not periodic), and w = 1 / (TV + eps) with
  eps = tv_eps_rel * sigma * N^2 * K;
* stage 2 uses the Wiener gain W = b^2 / (b^2 + sigma^2) of the pilot
  spectrum b applied to the noisy spectrum, with W = 1 at the 3-D DC, and the
  group weight 1 / sum(W^2); matching runs on the uint16-quantised first
  estimate Q = floor(clip(Y_b, 0, 1) * 65535 + 1/2).

Every floating-point quantity is float64; distances are exact int64.
"""
from __future__ import annotations

from dataclasses import dataclass, replace

import numpy as np

U16_MAX = 65535.0


@dataclass(frozen=True)
class Params:
    patch: int = 8          # N (block side)
    step: int = 3           # reference grid step
    search: int = 39        # odd search window side S; displacements in [-S//2, S//2]
    k_ht: int = 16          # group size, stage 1
    k_wiener: int = 32      # group size, stage 2
    ht_a: float = 3.6       # tau_l = sigma * (ht_a - ht_b * l)   (Sec. 5)
    ht_b: float = 0.3
    ht_weight: str = "tv"   # "tv" (Sec. 3.1), "nnz" or "unit"
    tv_eps_rel: float = 1e-3
    keep_dc: bool = True

    def with_(self, **kw) -> "Params":
        return replace(self, **kw)


DEFAULT = Params()


# ---------------------------------------------------------------------------
# Notation: periodic blocks (Sec. 1.2)
# ---------------------------------------------------------------------------

def reference_grid(H: int, W: int, step: int):
    """Reference top-left rows and columns; references are their Cartesian
    product in raster order (row index outer)."""
    return np.arange(0, H, step), np.arange(0, W, step)


def n_refs(H: int, W: int, step: int) -> int:
    ys, xs = reference_grid(H, W, step)
    return len(ys) * len(xs)


def displacements(search: int):
    """All (dy, dx) of the search window in rank order r = (dy+R)*S + (dx+R)."""
    R = search // 2
    d = np.arange(-R, R + 1)
    dy, dx = np.meshgrid(d, d, indexing="ij")
    return dy.ravel(), dx.ravel()


def block(Z: np.ndarray, i: int, j: int, N: int) -> np.ndarray:
    """z^{ij}[a, b] = Z[(i + a) mod H, (j + b) mod W]  (eq. (1) and Fblock)."""
    H, W = Z.shape
    return Z[np.ix_((i + np.arange(N)) % H, (j + np.arange(N)) % W)]


def _blocks(Z: np.ndarray, ys: np.ndarray, xs: np.ndarray, N: int) -> np.ndarray:
    """Blocks with top-left (ys[g], xs[g]) -> array [G, N, N]."""
    H, W = Z.shape
    a = np.arange(N)
    rows = (ys[:, None] + a[None, :]) % H            # [G, N]
    cols = (xs[:, None] + a[None, :]) % W
    return Z[rows[:, :, None], cols[:, None, :]]


# ---------------------------------------------------------------------------
# Block matching (Sec. 2, eq. dfg; Sec. 3.1 arg_K min)
# ---------------------------------------------------------------------------

def block_distances(Z: np.ndarray, ref_y: np.ndarray, ref_x: np.ndarray,
                    N: int, search: int) -> np.ndarray:
    """d[g, r] = ||z^{ref_g} - z^{ref_g + delta_r}||^2 in exact int64 (eq. dfg),
    for every displacement delta_r of the search window."""
    Zi = Z.astype(np.int64)
    dys, dxs = displacements(search)
    ref = _blocks(Zi, ref_y, ref_x, N)
    out = np.empty((len(ref_y), len(dys)), dtype=np.int64)
    for r, (dy, dx) in enumerate(zip(dys, dxs)):
        cand = _blocks(Zi, ref_y + dy, ref_x + dx, N)
        out[:, r] = ((ref - cand) ** 2).sum(axis=(1, 2))
    return out


def select_matches(dist: np.ndarray, K: int, search: int) -> np.ndarray:
    """arg_K min: slot 0 is the reference itself (zero displacement); slots
    1..K-1 are the K-1 smallest (distance, rank) keys among the other
    displacements, in ascending key order (lower rank wins ties)."""
    G, S2 = dist.shape
    r0 = S2 // 2
    ranks = np.arange(S2, dtype=np.int64)
    keys = dist * np.int64(1 << 11) + ranks[None, :]
    keys[:, r0] = np.iinfo(np.int64).max
    best = np.sort(keys, axis=1)[:, :K - 1]
    idx = np.empty((G, K), dtype=np.int64)
    idx[:, 0] = r0
    idx[:, 1:] = best & ((1 << 11) - 1)
    return idx


def ref_coords(H: int, W: int, step: int, ref_ids=None):
    ys, xs = reference_grid(H, W, step)
    ry = np.repeat(ys, len(xs))
    rx = np.tile(xs, len(ys))
    if ref_ids is not None:
        ref_ids = np.asarray(ref_ids)
        ry, rx = ry[ref_ids], rx[ref_ids]
    return ry, rx


def match(Z: np.ndarray, K: int, params: Params = DEFAULT, ref_ids=None) -> np.ndarray:
    """Displacement ranks idx[g, k] of the K matched blocks of each reference."""
    H, W = Z.shape
    ry, rx = ref_coords(H, W, params.step, ref_ids)
    d = block_distances(Z, ry, rx, params.patch, params.search)
    return select_matches(d, K, params.search)


def match_positions(H, W, idx, ry, rx, search):
    """Top-left (y, x) of every matched block, [G, K] each (periodic)."""
    R = search // 2
    dy = idx // search - R
    dx = idx % search - R
    return (ry[:, None] + dy) % H, (rx[:, None] + dx) % W


# ---------------------------------------------------------------------------
# Transforms (Sec. 5 parameter list: bior1.5, Haar, 3 levels; Sec. 4: DCT)
# ---------------------------------------------------------------------------

# Analysis low-pass of the biorthogonal spline pair of order 1.5 (Cohen,
# Daubechies and Feauveau): synthesis scaling function is the Haar box, the
# analysis filter has five zeros at the Nyquist frequency.  Taps at offsets
# -4 .. 5 relative to 2n.
BIOR15_LO = np.sqrt(2.0) / 256.0 * np.array([3, -3, -22, 22, 128, 128, 22, -22, -3, 3], dtype=np.float64)
BIOR15_OFFSETS = np.arange(-4, 6)


def bior15_analysis_matrix(L: int) -> np.ndarray:
    """One periodic analysis level on a length-L signal (L even):
    rows 0..L/2-1: a[n] = sum_i h_i x[(2n+i) mod L]; rows L/2..L-1:
    d[n] = (x[2n+1] - x[2n]) / sqrt(2)."""
    A = np.zeros((L, L))
    for n in range(L // 2):
        for h, off in zip(BIOR15_LO, BIOR15_OFFSETS):
            A[n, (2 * n + off) % L] += h
        A[L // 2 + n, 2 * n] = -1.0 / np.sqrt(2.0)
        A[L // 2 + n, 2 * n + 1] = 1.0 / np.sqrt(2.0)
    return A


def _levels(N: int) -> int:
    return int(np.log2(N))


def bior2d_forward(P: np.ndarray) -> np.ndarray:
    """Periodic 2-D Mallat decomposition to full depth (3 levels for N = 8):
    each level applies the 1-D analysis step to the rows and columns of the
    current low-low block.  P: [..., N, N]."""
    X = np.array(P, dtype=np.float64, copy=True)
    L = X.shape[-1]
    while L >= 2:
        A = bior15_analysis_matrix(L)
        X[..., :L, :L] = A @ X[..., :L, :L] @ A.T
        L //= 2
    return X


def bior2d_inverse(C: np.ndarray) -> np.ndarray:
    X = np.array(C, dtype=np.float64, copy=True)
    N = X.shape[-1]
    L = 2
    while L <= N:
        Ai = np.linalg.inv(bior15_analysis_matrix(L))
        X[..., :L, :L] = Ai @ X[..., :L, :L] @ Ai.T
        L *= 2
    return X


def bior2d_matrix(N: int = 8) -> np.ndarray:
    """The 2-D forward transform as an (N*N) x (N*N) matrix on row-major blocks."""
    E = np.eye(N * N).reshape(N * N, N, N)
    return bior2d_forward(E).reshape(N * N, N * N).T


def coefficient_level(N: int = 8) -> np.ndarray:
    """Wavelet level of each 2-D Mallat coefficient: finest details are level
    1, the approximation belongs to the coarsest level log2(N)."""
    J = _levels(N)
    lev = np.zeros((N, N), dtype=np.int64)
    for u in range(N):
        for v in range(N):
            m = max(u, v)
            lev[u, v] = J if m == 0 else J - int(np.floor(np.log2(m)))
    return lev


def dct_matrix(N: int = 8) -> np.ndarray:
    """Orthonormal DCT-II: C[k, n] = alpha_k cos(pi (2n+1) k / (2N))."""
    k = np.arange(N)[:, None]
    n = np.arange(N)[None, :]
    C = np.cos(np.pi * (2 * n + 1) * k / (2 * N))
    C[0, :] *= np.sqrt(1.0 / N)
    C[1:, :] *= np.sqrt(2.0 / N)
    return C


def dct2d_forward(P: np.ndarray) -> np.ndarray:
    C = dct_matrix(P.shape[-1])
    return C @ P @ C.T


def dct2d_inverse(X: np.ndarray) -> np.ndarray:
    C = dct_matrix(X.shape[-1])
    return C.T @ X @ C


def haar_matrix(K: int) -> np.ndarray:
    """Orthonormal full-depth Haar transform along a length-K group axis (K a
    power of two).  Row 0 is the normalised sum; the other rows are the
    (x0 - x1)/sqrt(2) differences of each level, finest level last."""
    if K == 1:
        return np.ones((1, 1))
    half = haar_matrix(K // 2)
    pair_sum = np.array([[1.0, 1.0]]) / np.sqrt(2.0)
    pair_diff = np.array([[1.0, -1.0]]) / np.sqrt(2.0)
    top = np.kron(half, pair_sum)
    bottom = np.kron(np.eye(K // 2), pair_diff)
    return np.vstack([top, bottom])


def haar_forward(G: np.ndarray) -> np.ndarray:
    """Haar along axis 1 of [G, K, ...]."""
    Hk = haar_matrix(G.shape[1])
    return np.einsum("jk,gk...->gj...", Hk, G)


def haar_inverse(G: np.ndarray) -> np.ndarray:
    Hk = haar_matrix(G.shape[1])
    return np.einsum("jk,gj...->gk...", Hk, G)


# ---------------------------------------------------------------------------
# Stage 1: hard-threshold collaborative filtering (Sec. 3.1, Sec. 5)
# ---------------------------------------------------------------------------

def ht_thresholds(sigma: float, params: Params = DEFAULT) -> np.ndarray:
    """tau(u, v) = sigma * (a - b * level(u, v))  (Sec. 5)."""
    lev = coefficient_level(params.patch)
    return sigma * (params.ht_a - params.ht_b * lev)


def hard_threshold(C: np.ndarray, tau: np.ndarray) -> np.ndarray:
    """Upsilon(alpha) = alpha if |alpha| >= lambda, else 0 (Sec. 3.1)."""
    return np.where(np.abs(C) >= tau, C, 0.0)


def ht_filter_groups(P: np.ndarray, sigma: float, params: Params = DEFAULT):
    """Filter groups P [G, K, N, N] (values on the [0, 1] scale).

    Returns (U, w, margin): filtered groups, aggregation weights, and for each
    group the smallest relative distance | |C| - tau | / tau over the
    coefficients whose keep/kill decision the threshold takes (used by the
    parity protocol to flag decisions that float32 cannot reproduce)."""
    G, K, N, _ = P.shape
    C = haar_forward(bior2d_forward(P))                       # [G, K, N, N]
    tau = np.array(np.broadcast_to(ht_thresholds(sigma, params), C.shape))
    decided = np.ones(C.shape, dtype=bool)
    if params.keep_dc:
        tau[:, 0, 0, 0] = 0.0                                 # the 3-D DC is never shrunk
        decided[:, 0, 0, 0] = False
    Chat = hard_threshold(C, tau)
    keep = np.abs(C) >= tau                                   # retained coefficients (for "nnz")
    with np.errstate(divide="ignore", invalid="ignore"):
        rel = np.abs(np.abs(C) - tau) / np.where(tau > 0, tau, 1.0)
    rel = np.where(decided & (tau > 0), rel, np.inf)
    margin = rel.reshape(G, -1).min(axis=1)
    U = bior2d_inverse(haar_inverse(Chat))
    if params.ht_weight == "tv":
        tv = (np.abs(np.diff(U, axis=1)).sum(axis=(1, 2, 3))
              + np.abs(np.diff(U, axis=2)).sum(axis=(1, 2, 3))
              + np.abs(np.diff(U, axis=3)).sum(axis=(1, 2, 3)))
        eps = params.tv_eps_rel * sigma * N * N * K
        w = 1.0 / (tv + eps)
    elif params.ht_weight == "nnz":
        w = 1.0 / np.maximum(keep.reshape(G, -1).sum(axis=1), 1)
    elif params.ht_weight == "unit":
        w = np.ones(G)
    else:
        raise ValueError(params.ht_weight)
    return U, w, margin


# ---------------------------------------------------------------------------
# Stage 2: empirical Wiener collaborative filtering (Sec. 4)
# ---------------------------------------------------------------------------

def wiener_filter_groups(Pn: np.ndarray, Pp: np.ndarray, sigma: float):
    """Noisy groups Pn and pilot groups Pp [G, K, N, N] -> (U, w)."""
    p = haar_forward(dct2d_forward(Pn))
    b = haar_forward(dct2d_forward(Pp))
    Wt = b * b / (b * b + sigma * sigma)
    Wt[:, 0, 0, 0] = 1.0
    U = dct2d_inverse(haar_inverse(Wt * p))
    w = 1.0 / (Wt * Wt).sum(axis=(1, 2, 3))
    return U, w


# ---------------------------------------------------------------------------
# Aggregation (Sec. 3.1: weighted average of the filtered blocks)
# ---------------------------------------------------------------------------

def aggregate(H: int, W: int, U: np.ndarray, w: np.ndarray, py: np.ndarray, px: np.ndarray,
              num: np.ndarray | None = None, den: np.ndarray | None = None):
    """num[pos + (a, b)] += w_g U[g, k, a, b]; den[...] += w_g over every block
    of every group, with periodic positions.  py, px: [G, K] top-left corners."""
    G, K, N, _ = U.shape
    if num is None:
        num = np.zeros((H, W))
        den = np.zeros((H, W))
    a = np.arange(N)
    rows = (py[:, :, None, None] + a[None, None, :, None]) % H     # [G, K, N, 1]
    cols = (px[:, :, None, None] + a[None, None, None, :]) % W     # [G, K, 1, N]
    rows = np.broadcast_to(rows, U.shape)
    cols = np.broadcast_to(cols, U.shape)
    wb = np.broadcast_to(w[:, None, None, None], U.shape)
    np.add.at(num, (rows, cols), wb * U)
    np.add.at(den, (rows, cols), wb)
    return num, den


def _chunks(n: int, size: int):
    for s in range(0, n, size):
        yield np.arange(s, min(n, s + size))


def refs_for_window(H, W, params: Params, y0, x0, h, w):
    """Ids of every reference whose matched blocks can reach the window
    [y0, y0+h) x [x0, x0+w) (periodic)."""
    R = params.search // 2
    N = params.patch
    ys, xs = reference_grid(H, W, params.step)

    def near(coords, lo, n, M):
        # block rows [c + d, c + d + N) with |d| <= R intersect [lo, lo + n)
        off = (coords - (lo - R - N + 1)) % M
        return np.nonzero(off < n + 2 * R + N - 1)[0]

    py = near(ys, y0, h, H)
    qx = near(xs, x0, w, W)
    return (py[:, None] * len(xs) + qx[None, :]).ravel()


# ---------------------------------------------------------------------------
# Whole stages
# ---------------------------------------------------------------------------

def basic_estimate(Z: np.ndarray, sigma: float, params: Params = DEFAULT, ref_ids=None,
                   chunk: int = 4096, return_parts: bool = False):
    """Stage 1 (G-BM3D1) on uint16 Z.  Returns Y_b [H, W] float64 on the [0, 1]
    scale.  With ref_ids, only those references contribute (used to evaluate
    a window exactly: pass refs_for_window and read only that window).
    With return_parts, also returns (idx, margin, num, den)."""
    H, W = Z.shape
    z = Z.astype(np.float64) / U16_MAX
    ry_all, rx_all = ref_coords(H, W, params.step)
    ids = np.arange(len(ry_all)) if ref_ids is None else np.asarray(ref_ids)
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    idx_all = np.empty((len(ids), params.k_ht), dtype=np.int64)
    margin_all = np.empty(len(ids))
    for c in _chunks(len(ids), chunk):
        g = ids[c]
        ry, rx = ry_all[g], rx_all[g]
        idx = select_matches(block_distances(Z, ry, rx, params.patch, params.search),
                             params.k_ht, params.search)
        py, px = match_positions(H, W, idx, ry, rx, params.search)
        P = _blocks(z, py.ravel(), px.ravel(), params.patch).reshape(len(g), params.k_ht,
                                                                     params.patch, params.patch)
        U, w, margin = ht_filter_groups(P, sigma, params)
        aggregate(H, W, U, w, py, px, num, den)
        idx_all[c] = idx
        margin_all[c] = margin
    with np.errstate(divide="ignore", invalid="ignore"):
        Y = num / den
    if return_parts:
        return Y, (idx_all, margin_all, num, den)
    return Y


def quantize(Y: np.ndarray) -> np.ndarray:
    """Pilot quantisation Q = floor(clip(Y, 0, 1) * 65535 + 1/2) (NaN -> 0)."""
    Y = np.nan_to_num(np.asarray(Y, dtype=np.float64), nan=0.0)
    return np.floor(np.clip(Y, 0.0, 1.0) * U16_MAX + 0.5).astype(np.uint16)


def wiener_estimate(Z: np.ndarray, pilot: np.ndarray, sigma: float, params: Params = DEFAULT,
                    ref_ids=None, chunk: int = 2048, return_parts: bool = False):
    """Stage 2 on uint16 noisy Z with uint16 pilot (matching runs on the pilot)."""
    H, W = Z.shape
    z = Z.astype(np.float64) / U16_MAX
    q = pilot.astype(np.float64) / U16_MAX
    ry_all, rx_all = ref_coords(H, W, params.step)
    ids = np.arange(len(ry_all)) if ref_ids is None else np.asarray(ref_ids)
    num = np.zeros((H, W))
    den = np.zeros((H, W))
    idx_all = np.empty((len(ids), params.k_wiener), dtype=np.int64)
    K, N = params.k_wiener, params.patch
    for c in _chunks(len(ids), chunk):
        g = ids[c]
        ry, rx = ry_all[g], rx_all[g]
        idx = select_matches(block_distances(pilot, ry, rx, N, params.search), K, params.search)
        py, px = match_positions(H, W, idx, ry, rx, params.search)
        Pn = _blocks(z, py.ravel(), px.ravel(), N).reshape(len(g), K, N, N)
        Pp = _blocks(q, py.ravel(), px.ravel(), N).reshape(len(g), K, N, N)
        U, w = wiener_filter_groups(Pn, Pp, sigma)
        aggregate(H, W, U, w, py, px, num, den)
        idx_all[c] = idx
    with np.errstate(divide="ignore", invalid="ignore"):
        Y = num / den
    if return_parts:
        return Y, (idx_all, num, den)
    return Y


def denoise(Z: np.ndarray, sigma: float, params: Params = DEFAULT):
    """Both stages (G-BM3D2).  Returns (Y, Y_b, Q)."""
    Yb = basic_estimate(Z, sigma, params)
    Q = quantize(Yb)
    Y = wiener_estimate(Z, Q, sigma, params)
    return Y, Yb, Q


def flagged_pixels(H: int, W: int, idx: np.ndarray, margin: np.ndarray, params: Params,
                   ref_ids=None, rel_tol: float = 1e-5) -> np.ndarray:
    """Mask of pixels covered by any block of a group holding a threshold
    decision within rel_tol of tau (float32 may decide those differently)."""
    ry, rx = ref_coords(H, W, params.step, ref_ids)
    sel = margin < rel_tol
    mask = np.zeros((H, W), dtype=bool)
    if not sel.any():
        return mask
    py, px = match_positions(H, W, idx[sel], ry[sel], rx[sel], params.search)
    a = np.arange(params.patch)
    rows = (py[:, :, None, None] + a[None, None, :, None]) % H
    cols = (px[:, :, None, None] + a[None, None, None, :]) % W
    rows, cols = np.broadcast_arrays(rows, cols)
    mask[rows, cols] = True
    return mask


def psnr(Y: np.ndarray, clean: np.ndarray) -> float:
    """10 log10(1 / MSE) of clip(Y, 0, 1) against the clean image."""
    mse = np.mean((np.clip(Y, 0.0, 1.0) - clean) ** 2)
    return float(10.0 * np.log10(1.0 / mse))
