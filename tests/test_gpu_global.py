"""Global stage 1 (volume form) through the C ABI against the CPU oracle.

Bars: tile matches bit-exact; the estimate within max-abs 2e-4 of the
oracle and within 0.01 dB PSNR.  (A volume coefficient lying within float32
rounding of its threshold could be kept on one side and dropped on the
other; none is in these seeded cases, whose largest difference is ~4e-7.)
The zero-threshold identity and constant images are exact to float32
rounding of the transforms.
"""
import sys

import numpy as np
import pytest

from oracle import gbm3d_oracle as O
from oracle import global_oracle as GO
from paper_2103_10765_amd import synth

pytestmark = pytest.mark.gpu

SIG = 25.0 / 255.0


def say(*a):
    print(*a, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def torch():
    import torch as t
    if not t.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    return t


@pytest.fixture(scope="module")
def G(torch):
    from paper_2103_10765_amd import gbm3d
    return gbm3d


@pytest.fixture(scope="module")
def ctx(G):
    c = G.Context(0)
    yield c
    c.close()


def up(torch, a):
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def oparams(gp):
    return GO.GDEFAULT.with_(patch=gp.patch, search=gp.search, k=gp.k, levels=gp.levels, cycles=gp.cycles,
                             shifts=tuple(gp.shifts[i] for i in range(gp.n_shifts)), ht_a=gp.ht_a, ht_b=gp.ht_b)


CASES = [
    # H, W, sigma*255, seed, overrides
    (64, 80, 25, 21, {}),
    (128, 128, 15, 22, {}),
    (96, 112, 50, 23, {}),
    (48, 64, 25, 24, {"patch": 8, "search": 15, "k": 8, "levels": 2, "cycles": 1, "shifts": (0,)}),
    (64, 64, 25, 25, {"k": 32, "search": 39, "shifts": (0, 4, 8)}),
    # several cycle spins filtered in the same launches
    (64, 48, 25, 26, {"cycles": 4, "levels": 1, "shifts": (0, 2)}),
    (48, 80, 35, 27, {"cycles": 3, "shifts": (0, 4, 8, 12)}),
]


@pytest.mark.parametrize("H,W,s,seed,ov", CASES)
def test_global_match_parity(torch, G, ctx, H, W, s, seed, ov):
    say("global match", H, W, ov)
    _, Z = synth.make_case(H, W, s / 255, seed)
    gp = G.global_default_params(**ov)
    idx = ctx.global_match(up(torch, Z), gp).cpu().numpy().astype(np.int64)
    assert np.array_equal(idx, GO.match_tiles(Z, oparams(gp)))


@pytest.mark.parametrize("H,W,s,seed,ov", CASES)
def test_global_parity(torch, G, ctx, H, W, s, seed, ov):
    say("global basic", H, W, s, ov)
    clean, Z = synth.make_case(H, W, s / 255, seed)
    gp = G.global_default_params(**ov)
    Yg = ctx.global_basic(up(torch, Z), s / 255, gp).cpu().numpy().astype(np.float64)
    Yo = GO.global_basic(Z, s / 255, oparams(gp))
    err = np.abs(Yg - Yo)
    say("max", err.max(), "p99.9", np.quantile(err, 0.999), "psnr", O.psnr(Yg, clean), O.psnr(Yo, clean))
    assert err.max() <= 2e-4
    assert abs(O.psnr(Yg, clean) - O.psnr(Yo, clean)) <= 0.01


def test_global_zero_threshold_identity(torch, G, ctx):
    _, Z = synth.make_case(64, 96, SIG, 26)
    Yg = ctx.global_basic(up(torch, Z), SIG, G.global_default_params(ht_a=0.0, ht_b=0.0)).cpu().numpy()
    assert np.abs(Yg - Z / 65535.0).max() < 1e-5


def test_global_constant_image(torch, G, ctx):
    Z = np.full((48, 64), 41000, dtype=np.uint16)
    Yg = ctx.global_basic(up(torch, Z), SIG).cpu().numpy()
    assert np.abs(Yg - 41000 / 65535.0).max() < 2e-6


def test_global_full_size(torch, G, ctx):
    """512 x 512 (the benchmark image) against the oracle."""
    say("global basic 512")
    clean, Z = synth.single_image_case(512, SIG, 2)
    Yg = ctx.global_basic(up(torch, Z), SIG).cpu().numpy().astype(np.float64)
    Yo = GO.global_basic(Z, SIG)
    err = np.abs(Yg - Yo)
    say("max", err.max(), "p99.9", np.quantile(err, 0.999), "psnr", O.psnr(Yg, clean), O.psnr(Yo, clean))
    assert err.max() <= 2e-4
    assert abs(O.psnr(Yg, clean) - O.psnr(Yo, clean)) <= 0.01


def test_global_rejects_bad_shapes(G, ctx, torch):
    """Sides below the search window are refused; the tile matching alone
    still needs multiples of the tile side."""
    with pytest.raises(G.GBM3DError):
        ctx.global_basic(up(torch, np.zeros((30, 64), dtype=np.uint16)), SIG)
    with pytest.raises(G.GBM3DError):
        ctx.global_match(up(torch, np.zeros((50, 64), dtype=np.uint16)))


@pytest.mark.parametrize("H,W,s,seed,ov", [(50, 64, 25, 28, {}), (70, 93, 25, 29, {}),
                                            (45, 61, 35, 30, {"patch": 8, "search": 15, "k": 8, "levels": 2})])
def test_global_parity_mirror_padded(torch, G, ctx, H, W, s, seed, ov):
    """Sides that are not multiples of the tile side: mirror padding at the
    bottom and right, filtering, cropping; against the oracle's."""
    say("global basic padded", H, W, s, ov)
    clean, Z = synth.make_case(H, W, s / 255, seed)
    gp = G.global_default_params(**ov)
    Yg = ctx.global_basic(up(torch, Z), s / 255, gp).cpu().numpy().astype(np.float64)
    Yo = GO.global_basic(Z, s / 255, oparams(gp))
    assert Yg.shape == (H, W)
    err = np.abs(Yg - Yo)
    say("max", err.max(), "psnr", O.psnr(Yg, clean), O.psnr(Yo, clean))
    assert err.max() <= 2e-4
    assert abs(O.psnr(Yg, clean) - O.psnr(Yo, clean)) <= 0.01
