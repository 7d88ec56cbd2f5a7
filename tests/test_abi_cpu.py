"""CPU checks of the C ABI: the library loads, exports every entry point that
include/gbm3d.h declares, and validates arguments on the host without a GPU."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "gbm3d.h")


def _declared():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(gbm3d_\w+)\s*\(", src)))


@pytest.fixture(scope="module")
def G():
    from paper_2103_10765_amd import gbm3d
    if not os.path.exists(gbm3d.LIB_PATH):
        pytest.fail("libgbm3d.so is not built (run __graft_entry__.build())")
    return gbm3d


def test_every_declared_symbol_is_exported(G):
    names = _declared()
    assert len(names) >= 12
    L = G.lib()
    missing = [n for n in names if not hasattr(L, n)]
    assert not missing, missing
    # and the binding declares a signature for each
    assert set(names) <= set(G._SIGNATURES), set(names) - set(G._SIGNATURES)


def test_default_params(G):
    p = G.default_params()
    assert p.struct_size == ctypes.sizeof(G.Params)
    assert (p.patch, p.step, p.search, p.k_ht, p.k_wiener) == (8, 3, 39, 16, 32)
    assert p.ht_source == G.HT_STACK
    assert abs(p.ht_a - 3.6) < 1e-6 and abs(p.ht_b - 0.3) < 1e-6
    assert p.ht_weight == G.W_TV and p.keep_dc == 1
    assert p.bm_split == 0 and p.bm_method == G.BM_AUTO


def test_status_strings_and_version(G):
    L = G.lib()
    assert L.gbm3d_status_str(0) == b"ok"
    assert L.gbm3d_status_str(G.EINVAL) == b"invalid argument"
    assert b"gfx950" in L.gbm3d_version()


@pytest.mark.parametrize("H,W,step,n", [(512, 512, 3, 171 * 171), (128, 128, 3, 43 * 43), (40, 41, 3, 14 * 14),
                                        (0, 5, 3, 0)])
def test_n_refs(G, H, W, step, n):
    assert G.n_refs(H, W, step) == n


def test_validation_rules(G):
    s25 = 25 / 255
    assert G.check_args(512, 512, s25) == G.OK
    assert G.check_args(39, 39, s25) == G.OK
    assert G.check_args(38, 512, s25) == G.EINVAL            # below the search window
    assert G.check_args(512, 32769, s25) == G.EINVAL
    assert G.check_args(512, 512, 0.0) == G.EINVAL
    assert G.check_args(512, 512, float("nan")) == G.EINVAL
    assert G.check_args(512, 512, float("inf")) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(search=38)) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(search=41)) == G.EINVAL
    assert G.check_args(16, 16, s25, G.default_params(search=15)) == G.OK
    assert G.check_args(512, 512, s25, G.default_params(k_ht=12)) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(k_wiener=64)) == G.EINVAL
    assert G.check_args(64, 64, s25, G.default_params(search=3, k_wiener=16)) == G.EINVAL  # K > search^2
    assert G.check_args(512, 512, s25, G.default_params(patch=16)) == G.EUNSUPPORTED
    assert G.check_args(512, 512, s25, G.default_params(step=4)) == G.EUNSUPPORTED
    assert G.check_args(512, 512, s25, G.default_params(ht_weight=7)) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(tv_eps_rel=-1.0)) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(tv_eps_rel=0.0)) == G.EINVAL
    for m in (G.BM_AUTO, G.BM_SHIFT, G.BM_CORR):
        assert G.check_args(512, 512, s25, G.default_params(bm_method=m)) == G.OK
    assert G.check_args(512, 512, s25, G.default_params(bm_method=3)) == G.EINVAL
    assert G.check_args(512, 512, s25, G.default_params(bm_split=3)) == G.EINVAL
    p = G.default_params()
    p.struct_size = 4
    assert G.check_args(512, 512, s25, p) == G.EINVAL
    assert "struct_size" in G.last_thread_error()


def test_null_context_is_rejected(G):
    L = G.lib()
    assert L.gbm3d_basic(None, None, 64, 64, 0.1, None, None, None) == G.EINVAL
    assert L.gbm3d_denoise(None, None, 64, 64, 0.1, None, None, None, None, None) == G.EINVAL
    assert "ctx" in G.last_thread_error()
    assert L.gbm3d_autotune(None, None, 64, 64, 16, None, 1, None, None, None, None) == G.EINVAL
    assert L.gbm3d_tune_load(None, b"/nonexistent") == G.EINVAL
    assert L.gbm3d_tune_save(None, b"/nonexistent") == G.EINVAL


def test_create_without_device_fails_cleanly(G):
    import torch
    if torch.cuda.is_available():
        pytest.skip("a GPU is present")
    h = ctypes.c_void_p()
    s = G.lib().gbm3d_create(ctypes.byref(h), 0)
    assert s in (G.EHIP, G.EINVAL) and not h.value


def test_probe_operation_counts(G):
    """Arithmetic operations of a peak-rate probe launch: 8 chains per thread
    (fp64 FMA) or per wave (one 16x16x64 int8 / 16x16x32 bf16 MFMA each), a
    multiply-add counting 2; unknown kinds give 0."""
    L = G.lib()
    blocks, iters = 3, 5
    threads, waves = blocks * 256, blocks * 4
    assert L.gbm3d_probe_ops(G.PROBE_FP64, blocks, iters) == threads * iters * 8 * 2
    assert L.gbm3d_probe_ops(G.PROBE_MFMA_I8, blocks, iters) == waves * iters * 8 * 16 * 16 * 64 * 2
    assert L.gbm3d_probe_ops(G.PROBE_MFMA_BF16, blocks, iters) == waves * iters * 8 * 16 * 16 * 32 * 2
    assert L.gbm3d_probe_ops(7, blocks, iters) == 0.0
