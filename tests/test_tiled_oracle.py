"""Pins of the sub-image form of the oracle (Sec. 5, 256 + N sub-images)."""
import numpy as np
import pytest

from oracle import gbm3d_oracle as O
from oracle import tiled_oracle as T
from paper_2103_10765_amd import synth


@pytest.mark.parametrize("L,size,stride", [(1000, 264, 256), (600, 264, 256), (513, 264, 256), (265, 264, 256),
                                           (264, 264, 256), (100, 264, 256), (300, 72, 64), (96, 56, 48)])
def test_plan_partitions_the_axis_by_nearest_centre(L, size, stride):
    """The owned ranges tile [0, L) in order; every sub-image lies in [0, L),
    starts at most `stride` after the previous one, the first at 0 and the
    last flush with the end; and every pixel is owned by a covering sub-image
    whose centre is nearest to it (brute force over all covering ones)."""
    plan = T.axis_plan(L, size, stride)
    assert plan[0][0] == 0 and plan[0][2] == 0 and plan[-1][3] == L
    assert plan[-1][0] + plan[-1][1] == L
    for (s, side, lo, hi), nxt in zip(plan, plan[1:] + [None]):
        assert 0 <= s and s + side <= L and s <= lo < hi <= s + side
        if nxt is not None:
            assert nxt[2] == hi and 0 < nxt[0] - s <= stride
    for y in range(L):
        owner = [i for i, (s, side, lo, hi) in enumerate(plan) if lo <= y < hi]
        assert len(owner) == 1
        cover = [(abs(y + 0.5 - (s + side / 2.0)), i) for i, (s, side, _, _) in enumerate(plan) if s <= y < s + side]
        best = min(d for d, _ in cover)
        assert abs(y + 0.5 - (plan[owner[0]][0] + plan[owner[0]][1] / 2.0)) <= best + 0.5


def test_one_sub_image_is_the_whole_image():
    clean, Z = synth.make_case(48, 56, 25 / 255, 31)
    Y, Yb, Q = T.denoise(Z, 25 / 255, size=64, stride=48)
    Yw, Ybw, Qw = O.denoise(Z, 25 / 255)
    assert np.array_equal(Y, Yw) and np.array_equal(Yb, Ybw) and np.array_equal(Q, Qw)


def test_constant_image_stays_constant():
    Z = np.full((70, 60), 30000, dtype=np.uint16)
    Y, Yb, _ = T.denoise(Z, 20 / 255, size=48, stride=40)
    assert np.allclose(Yb, 30000 / 65535, atol=1e-9) and np.allclose(Y, 30000 / 65535, atol=1e-9)


def test_stitched_pixels_come_from_their_sub_image():
    """Every stitched basic-estimate pixel equals that pixel of the stage-1
    estimate of the sub-image that owns it (computed here directly)."""
    _, Z = synth.make_case(60, 50, 25 / 255, 32)
    _, Yb, _ = T.denoise(Z, 25 / 255, size=40, stride=24)
    for (y0, h, ylo, yhi) in T.axis_plan(60, 40, 24):
        for (x0, w, xlo, xhi) in T.axis_plan(50, 40, 24):
            sub = O.basic_estimate(Z[y0:y0 + h, x0:x0 + w], 25 / 255)
            y, x = (ylo + yhi) // 2, (xlo + xhi) // 2
            assert Yb[y, x] == sub[y - y0, x - x0]
