"""The sub-image driver (Sec. 5, 256 + N sub-images) on the GPU: the same plan
as the oracle's sub-image form, every stitched pixel equal to the library's
own single-image call on its sub-image, and both stages within 0.01 dB PSNR
of the oracle's sub-image form."""
import numpy as np
import pytest

from oracle import gbm3d_oracle as O
from oracle import tiled_oracle as T
from paper_2103_10765_amd import synth

pytestmark = pytest.mark.gpu

PSNR_TOL = 0.01


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    from paper_2103_10765_amd import gbm3d
    c = gbm3d.Context(0)
    yield c
    c.close()


def test_plans_agree():
    from paper_2103_10765_amd import tiled
    for L, size, stride in ((4096, 264, 256), (512, 264, 256), (1000, 264, 256), (513, 264, 256), (200, 264, 256),
                            (96, 56, 48), (130, 72, 64)):
        assert [tuple(r) for r in tiled.sub_ranges(L, size, stride)] == [tuple(r) for r in T.axis_plan(L, size, stride)]


@pytest.mark.parametrize("H,W,size,stride,s255,seed", [(96, 88, 56, 48, 25, 41), (130, 70, 72, 64, 15, 42),
                                                       (120, 136, 48, 40, 50, 43)])
def test_tiled_parity(ctx, H, W, size, stride, s255, seed):
    import torch
    from paper_2103_10765_amd import tiled
    sigma = s255 / 255.0
    print("tiled", H, W, size, stride, s255, flush=True)
    clean, Z = synth.make_case(H, W, sigma, seed)
    Zt = torch.from_numpy(Z).cuda()
    out, basic, pilot = tiled.denoise(ctx, Zt, sigma, size=size, stride=stride)
    torch.cuda.synchronize()
    out_h, basic_h, pilot_h = out.cpu().numpy(), basic.cpu().numpy(), pilot.cpu().numpy()
    # the pilot is the stitched estimate quantised
    assert np.array_equal(pilot_h, O.quantize(basic_h.astype(np.float64)))
    # every owned pixel is the single-image call's on its sub-image, bit for bit
    for (y0, h, ya, yb) in T.axis_plan(H, size, stride):
        for (x0, w, xa, xb) in T.axis_plan(W, size, stride):
            sub = Zt[y0:y0 + h, x0:x0 + w].contiguous()
            b = ctx.basic(sub, sigma).cpu().numpy()
            assert np.array_equal(basic_h[ya:yb, xa:xb], b[ya - y0:yb - y0, xa - x0:xb - x0])
            o = ctx.wiener(sub, pilot[y0:y0 + h, x0:x0 + w].contiguous(), sigma).cpu().numpy()
            assert np.array_equal(out_h[ya:yb, xa:xb], o[ya - y0:yb - y0, xa - x0:xb - x0])
    # against the oracle's sub-image form
    Yo, Ybo, _ = T.denoise(Z, sigma, size=size, stride=stride)
    assert abs(O.psnr(basic_h.astype(np.float64), clean) - O.psnr(Ybo, clean)) <= PSNR_TOL
    assert abs(O.psnr(out_h.astype(np.float64), clean) - O.psnr(Yo, clean)) <= PSNR_TOL


def test_one_sub_image_is_the_whole_image(ctx):
    import torch
    from paper_2103_10765_amd import tiled
    _, Z = synth.make_case(72, 80, 25 / 255, 44)
    Zt = torch.from_numpy(Z).cuda()
    out, _, _ = tiled.denoise(ctx, Zt, 25 / 255)   # 264 > 80: one sub-image
    assert np.array_equal(out.cpu().numpy(), ctx.denoise(Zt, 25 / 255).cpu().numpy())
