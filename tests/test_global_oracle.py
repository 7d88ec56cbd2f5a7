"""Pins of the global stage-1 oracle (CPU only): transform round trip and
separability, band levels, brute-force tile matching, the volume's first
slice, zero-threshold identity, constants, and the averaging operators."""
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
