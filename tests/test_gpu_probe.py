"""The peak-rate probes run on the GPU, write their sink and reject bad
arguments before any launch."""
import pytest

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def ctx():
    import torch
    if not torch.cuda.is_available():
        pytest.fail("no GPU visible to torch")
    from paper_2103_10765_amd import gbm3d
    c = gbm3d.Context(0)
    yield c
    c.close()


@pytest.mark.parametrize("kind", [0, 1, 2])
def test_probe_runs(ctx, kind):
    import torch
    sink = torch.full((4 * 256,), float("nan"), dtype=torch.float32, device="cuda")
    out, ops = ctx.probe(kind, 4, 16, sink=sink)
    torch.cuda.synchronize()
    assert ops > 0
    assert bool(torch.isfinite(out).all())


def test_probe_rejects_bad_arguments(ctx):
    """Host-side validation through the C ABI: nothing is launched, so a
    one-block sink serves every case."""
    import torch
    from paper_2103_10765_amd import gbm3d
    sink = torch.zeros(256, dtype=torch.float32, device="cuda")
    L = gbm3d.lib()
    for kind, blocks, iters in ((3, 1, 4), (-1, 1, 4), (0, 0, 4), (0, 1, 0), (0, (1 << 20) + 1, 4), (0, 1, (1 << 20) + 1)):
        assert L.gbm3d_probe(ctx._h, kind, blocks, iters, sink.data_ptr(), None) == -1  # GBM3D_EINVAL
    assert L.gbm3d_probe(ctx._h, 0, 1, 4, None, None) == -1
    torch.cuda.synchronize()
    assert float(sink.abs().sum()) == 0.0
