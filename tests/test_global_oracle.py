"""Pins of the global stage-1 oracle (CPU only): transform round trip and
separability, band levels, brute-force tile matching, the volume's first
slice, zero-threshold identity, constants, the averaging operators, the TV
weights in closed form, and the kept final approximation band."""
import numpy as np

from oracle import gbm3d_oracle as O
from oracle import global_oracle as G
from paper_2103_10765_amd import synth

SIG = 25.0 / 255.0


def test_dwt3_round_trip():
    V = np.random.default_rng(0).random((16, 32, 48))
    assert np.abs(G.idwt3(G.dwt3(V, 3), 3) - V).max() < 1e-12


def test_dwt3_one_level_is_separable():
    """One level on a separable volume f(k) g(y) h(x) is the product of the
    three 1-D steps: Haar along k, the bior1.5 step along y and x."""
    rng = np.random.default_rng(1)
    f, g, h = rng.random(8), rng.random(16), rng.random(24)
    V = f[:, None, None] * g[None, :, None] * h[None, None, :]
    C = G.dwt3(V, 1)
    s = 1.0 / np.sqrt(2.0)
    fk = np.concatenate([(f[0::2] + f[1::2]) * s, (f[0::2] - f[1::2]) * s])
    taps = O.BIOR15_LO

    def bior(x):
        L = len(x)
        a = [sum(t * x[(2 * n + o) % L] for t, o in zip(taps, O.BIOR15_OFFSETS)) for n in range(L // 2)]
        d = [(x[2 * n + 1] - x[2 * n]) * s for n in range(L // 2)]
        return np.array(a + d)

    want = fk[:, None, None] * bior(g)[None, :, None] * bior(h)[None, None, :]
    assert np.abs(C - want).max() < 1e-12


def test_band_levels():
    lev = G.coefficient_levels(16, 32, 64, 3)
    n = 16 * 32 * 64
    assert (lev == 1).sum() == n - n // 8
    assert (lev == 2).sum() == n // 8 - n // 64
    assert (lev == 3).sum() == n // 64 - n // 512
    assert (lev == 0).sum() == n // 512 and lev[0, 0, 0] == 0


def test_tile_matching_brute_force():
    _, Z = synth.make_case(32, 48, SIG, 3)
    p = G.GDEFAULT.with_(search=9, k=4)
    idx = G.match_tiles(Z, p)
    Zi = Z.astype(np.int64)
    ry, rx = G.tile_refs(32, 48, 16)
    for g in range(len(ry)):
        keys = []
        for r in range(81):
            dy, dx = r // 9 - 4, r % 9 - 4
            d = int(((O.block(Zi, ry[g], rx[g], 16) - O.block(Zi, ry[g] + dy, rx[g] + dx, 16)) ** 2).sum())
            if r != 40:
                keys.append((d, r))
        keys.sort()
        assert idx[g, 0] == 40 and list(idx[g, 1:]) == [r for _, r in keys[:3]]


def test_first_slice_is_the_image():
    _, Z = synth.make_case(32, 32, SIG, 4)
    z = Z / 65535.0
    V = G.build_volume(z, G.match_tiles(Z), G.GDEFAULT)
    assert np.array_equal(V[0], z)


def test_zero_threshold_is_identity():
    _, Z = synth.make_case(48, 64, SIG, 5)
    Y = G.global_basic(Z, SIG, G.GDEFAULT.with_(ht_a=0.0, ht_b=0.0))
    assert np.abs(Y - Z / 65535.0).max() < 1e-12


def test_constant_image():
    Z = np.full((32, 48), 30000, dtype=np.uint16)
    Y = G.global_basic(Z, SIG)
    assert np.abs(Y - 30000 / 65535.0).max() < 1e-12


def test_single_spin_and_translation():
    _, Z = synth.make_case(32, 32, SIG, 6)
    z = Z / 65535.0
    p = G.GDEFAULT.with_(cycles=1, shifts=(0,))
    V = G.build_volume(z, G.match_tiles(Z, p), p)
    lev = G.coefficient_levels(*V.shape, p.levels)
    tau = np.where(lev > 0, SIG * (p.ht_a - p.ht_b * lev), 0.0)
    U0 = G.idwt3(O.hard_threshold(G.dwt3(V, p.levels), tau), p.levels)
    assert np.abs(G.filter_volume(V, SIG, p) - U0).max() < 1e-15
    assert np.array_equal(G.global_basic(Z, SIG, p), G.phi(Z, SIG, p))


def test_global_beats_noise_and_matches_grouped_quality():
    clean, Z = synth.make_case(64, 80, SIG, 11)
    Yg = G.global_basic(Z, SIG)
    Yb = O.basic_estimate(Z, SIG)
    assert O.psnr(Yg, clean) > O.psnr(Z / 65535.0, clean) + 8.0
    assert O.psnr(Yg, clean) > O.psnr(Yb, clean) - 0.5


def test_mirror_pad_repeats_the_edge_then_mirrors():
    """Rows / columns past the end read the image backwards from its last
    row / column (explicit loop); sizes already multiples are unchanged."""
    Z = np.arange(5 * 7, dtype=np.uint16).reshape(5, 7)
    P = G.mirror_pad(Z, 4)
    assert P.shape == (8, 8)
    for y in range(8):
        for x in range(8):
            ys = y if y < 5 else 2 * 5 - 1 - y
            xs = x if x < 7 else 2 * 7 - 1 - x
            assert P[y, x] == Z[ys, xs]
    assert np.array_equal(G.mirror_pad(P, 4), P)


def test_non_multiple_sizes_keep_constants():
    """A constant image of a size that is not a multiple of the tile side
    comes back constant and of its own size."""
    Z = np.full((37, 45), 20000, dtype=np.uint16)
    p = G.GDEFAULT.with_(patch=8, search=9, k=8, levels=2, shifts=(0,))
    Y = G.global_basic(Z, 20 / 255, p)
    assert Y.shape == (37, 45)
    assert np.allclose(Y, 20000 / 65535, atol=1e-9)


def test_tv_weights_closed_form():
    """w = 1 / (TV + eps) per tile, TV the anisotropic L1 norm of forward,
    non-periodic differences along the match axis and both image axes
    (Sec. 3.1 weight 1/TV), on four tiles whose TV has a closed form: a
    horizontal ramp a*x gives K N (N-1) |a|, a vertical ramp b*y gives
    K N (N-1) |b|, per-slice offsets c_k give N^2 sum |c_{k+1} - c_k|, and
    their sum adds up (each difference runs along one axis)."""
    N, K = 4, 4
    p = G.GDEFAULT.with_(patch=N, k=K)
    sig = 0.2
    a, b, c = 0.03, -0.05, np.array([0.0, 0.4, 0.1, 0.7])
    yy, xx = np.meshgrid(np.arange(N), np.arange(N), indexing="ij")
    U = np.zeros((K, 2 * N, 2 * N))
    U[:, :N, :N] = 0.5 + a * xx                                        # tile 0 (raster order)
    U[:, :N, N:] = 0.2 + b * yy                                        # tile 1
    U[:, N:, :N] = c[:, None, None] + 0 * xx                           # tile 2
    U[:, N:, N:] = c[:, None, None] + a * xx + b * yy                  # tile 3
    ramp = K * N * (N - 1)
    dc = N * N * np.abs(np.diff(c)).sum()
    tv = np.array([ramp * abs(a), ramp * abs(b), dc, ramp * (abs(a) + abs(b)) + dc])
    eps = p.tv_eps_rel * sig * N * N * K
    assert np.allclose(G.tv_weights(U, sig, p), 1.0 / (tv + eps), rtol=1e-13, atol=0)


def test_final_approximation_is_kept_details_thresholded():
    """Detail bands are hard-thresholded at tau_l = sigma (3.6 - 0.3 l) and the
    final approximation band is kept whatever its size (the reading of the
    3-D transform's threshold rule, Sec. 3): a volume whose coefficients are
    all in the approximation band, every one below tau_3, comes back exactly;
    adding one level-2 detail coefficient just below tau_2 and one level-1
    coefficient just above tau_1 returns the volume without the first."""
    K, H, W = 16, 32, 32
    p = G.GDEFAULT.with_(cycles=1)
    sig = 0.1
    lev = G.coefficient_levels(K, H, W, p.levels)
    tau = lambda l: sig * (p.ht_a - p.ht_b * l)
    rng = np.random.default_rng(21)
    C = np.zeros((K, H, W))
    approx = lev == 0
    C[approx] = rng.uniform(0.2, 0.9, approx.sum()) * tau(3) * rng.choice([-1.0, 1.0], approx.sum())
    V = G.idwt3(C, p.levels)
    assert np.abs(G.filter_volume(V, sig, p) - V).max() < 1e-12
    C2 = C.copy()
    k2 = tuple(np.argwhere(lev == 2)[5])
    k1 = tuple(np.argwhere(lev == 1)[100])
    C2[k2] = 0.999 * tau(2)
    C2[k1] = -1.001 * tau(1)
    want = C2.copy()
    want[k2] = 0.0
    got = G.filter_volume(G.idwt3(C2, p.levels), sig, p)
    assert np.abs(got - G.idwt3(want, p.levels)).max() < 1e-12
