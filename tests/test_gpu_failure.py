"""Failure handling forced from the host: with the workspace allocation hook
armed (GBM3D_FAULT_ALLOC), a call that needs to grow the context workspace
returns GBM3D_ENOMEM with its reason, launches nothing (the output keeps its
sentinel), and the context works normally once the hook is disarmed."""
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


@pytest.mark.parametrize("entry", ["basic", "denoise", "batch"])
def test_allocation_failure_returns_enomem_and_launches_nothing(torch, G, entry):
    H, W, sigma = 96, 80, 25.0 / 255.0
    _, Z = synth.make_case(H, W, sigma, 21)
    Zt = torch.from_numpy(Z).cuda()
    ctx = G.Context(0)  # fresh: every workspace buffer still has to be allocated
    try:
        out = torch.full((H, W), -5.0, dtype=torch.float32, device="cuda")
        os.environ["GBM3D_FAULT_ALLOC"] = "1"
        try:
            with pytest.raises(G.GBM3DError) as e:
                if entry == "basic":
                    ctx.basic(Zt, sigma, out=out)
                elif entry == "denoise":
                    ctx.denoise(Zt, sigma, out=out)
                else:
                    ctx.denoise_batch([Zt], [sigma], outs=[out], graph=True)
        finally:
            del os.environ["GBM3D_FAULT_ALLOC"]
        say(entry, "->", e.value)
        assert e.value.status == G.ENOMEM
        assert "allocation failure injected" in str(e.value)
        torch.cuda.synchronize()
        assert bool((out == -5.0).all()), "the failed call wrote its output"
        # the same context recovers
        ref = G.Context(0)
        try:
            if entry == "basic":
                got, want = ctx.basic(Zt, sigma, out=out), ref.basic(Zt, sigma)
            else:
                got, want = ctx.denoise(Zt, sigma, out=out), ref.denoise(Zt, sigma)
            torch.cuda.synchronize()
            assert torch.equal(got, want)
        finally:
            ref.close()
    finally:
        ctx.close()
