"""gbm3d_denoise_noalloc: the two-stage denoise with every intermediate buffer
in the library's static per-device scratch.  Through the C ABI it must give
exactly what gbm3d_denoise gives (same kernels, deterministic fixed-point
aggregation), on consecutive calls of different sizes, without growing any
workspace (the allocation-failure hook is armed during its calls), and refuse
an image whose buffers do not fit the scratch."""
import ctypes
import os
import sys

import numpy as np
import pytest

from paper_2103_10765_amd import synth

pytestmark = pytest.mark.gpu


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


class _NoAlloc:
    """Arms the workspace allocation-failure hook: any attempt of the library
    to grow a context workspace returns GBM3D_ENOMEM."""

    def __enter__(self):
        self.prev = os.environ.get("GBM3D_FAULT_ALLOC")
        os.environ["GBM3D_FAULT_ALLOC"] = "1"

    def __exit__(self, *exc):
        if self.prev is None:
            del os.environ["GBM3D_FAULT_ALLOC"]
        else:
            os.environ["GBM3D_FAULT_ALLOC"] = self.prev


def _run_both(torch, G, ref_ctx, na_ctx, H, W, sigma, seed, params):
    say(f"noalloc case {H}x{W} sigma {sigma * 255:.1f}/255 seed {seed} method {params.bm_method}")
    _, Z = synth.make_case(H, W, sigma, seed)
    Zt = torch.from_numpy(Z).cuda()
    ref_b = torch.empty((H, W), dtype=torch.float32, device="cuda")
    ref_q = torch.empty((H, W), dtype=torch.uint16, device="cuda")
    ref = ref_ctx.denoise(Zt, sigma, params, basic_out=ref_b, q_out=ref_q)
    torch.cuda.synchronize()
    out = torch.full((H, W), -7.0, dtype=torch.float32, device="cuda")
    b = torch.full((H, W), -7.0, dtype=torch.float32, device="cuda")
    q = torch.zeros((H, W), dtype=torch.uint16, device="cuda")
    with _NoAlloc():
        na_ctx.denoise_noalloc(Zt, sigma, params, out=out, basic_out=b, q_out=q)
        torch.cuda.synchronize()
    assert torch.equal(out, ref), f"{H}x{W}: max |diff| {(out - ref).abs().max().item()}"
    assert torch.equal(b, ref_b)
    assert torch.equal(q, ref_q)
    # without the optional intermediate outputs (basic and pilot in the scratch too)
    out2 = torch.full((H, W), -7.0, dtype=torch.float32, device="cuda")
    with _NoAlloc():
        na_ctx.denoise_noalloc(Zt, sigma, params, out=out2)
        torch.cuda.synchronize()
    assert torch.equal(out2, ref)


def test_noalloc_equals_denoise_twice_then_smaller(torch, G):
    ref_ctx = G.Context(0)
    na_ctx = G.Context(0)  # a fresh context: its workspace has never grown
    try:
        p = G.default_params()
        _run_both(torch, G, ref_ctx, na_ctx, 512, 512, 25.0 / 255.0, 2, p)
        # a smaller, ragged image next: the scratch still holds the first call's contents
        p2 = G.default_params(bm_method=G.BM_SHIFT)
        _run_both(torch, G, ref_ctx, na_ctx, 97, 131, 15.0 / 255.0, 11, p2)
        p3 = G.default_params(ht_source=G.HT_RECOMPUTE, search=21, k_ht=8, k_wiener=16)
        _run_both(torch, G, ref_ctx, na_ctx, 64, 200, 50.0 / 255.0, 12, p3)
    finally:
        ref_ctx.close()
        na_ctx.close()


def test_noalloc_rejects_images_beyond_the_scratch(torch, G):
    ctx = G.Context(0)
    try:
        H = W = 1024
        Zt = torch.zeros((H, W), dtype=torch.uint16, device="cuda")
        out = torch.full((H, W), -7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(G.GBM3DError) as e:
            ctx.denoise_noalloc(Zt, 0.1, out=out)
        assert e.value.status == G.EINVAL
        assert "scratch" in str(e.value)
        torch.cuda.synchronize()
        assert bool((out == -7.0).all()), "a rejected call wrote its output"
    finally:
        ctx.close()


def test_noalloc_size_limit(torch, G):
    """With the default parameters the largest square image whose buffers
    (basic estimate and pilot included) fit the scratch is 551 x 551: it runs
    and equals gbm3d_denoise; 552 x 552 is refused before any launch."""
    ref_ctx = G.Context(0)
    na_ctx = G.Context(0)
    try:
        _run_both(torch, G, ref_ctx, na_ctx, 551, 551, 25.0 / 255.0, 5, G.default_params())
        H = W = 552
        Zt = torch.zeros((H, W), dtype=torch.uint16, device="cuda")
        out = torch.full((H, W), -7.0, dtype=torch.float32, device="cuda")
        with pytest.raises(G.GBM3DError) as e:
            na_ctx.denoise_noalloc(Zt, 0.1, out=out)
        assert e.value.status == G.EINVAL
        torch.cuda.synchronize()
        assert bool((out == -7.0).all()), "a rejected call wrote its output"
    finally:
        ref_ctx.close()
        na_ctx.close()
