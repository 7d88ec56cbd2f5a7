"""Host-side logic of bench.py (no GPU): the algorithmic work each kernel is
priced with, the copy-calibrated counter traffic and the instruction counts
read from the committed summaries (each guarded by a digest of the kernel's
sources), and the one-GPU guard.  The benchmark line's roofline fractions are
computed from these."""
import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)
import bench  # noqa: E402

N512 = 171 * 171  # references on the step-3 grid of a 512 x 512 image


def test_matcher_work_is_five_ops_per_pixel_and_displacement():
    assert bench.algorithmic_work(512, 512, 39, 16, 32)["bm"] == ("alu", 5 * 512 * 512 * (39 * 39 - 1), "FLOP")


def test_group_and_reduce_bytes():
    H = W = 512
    w = bench.algorithmic_work(H, W, 39, 16, 32)
    # K spectra of 256 B gathered, K 2-byte ranks, K 8-byte weight atomics per
    # reference, the image's 8-byte numerator sums added into once
    assert w["group_ht"] == ("hbm", N512 * (16 * 256 + 2 * 16 + 8 * 16) + H * W * 8, "B")
    assert w["group_wiener"] == ("hbm", N512 * (2 * 32 * 256 + 2 * 32 + 8 * 32) + H * W * 8, "B")
    # numerator sums and block-start weights read, f32 estimate and u16 pilot written
    assert w["reduce"] == ("hbm", H * W * (8 + 8 + 4 + 2), "B")


def test_norm_tables_move_into_the_stack_launches():
    a = bench.algorithmic_work(512, 512, 39, 16, 32)
    b = bench.algorithmic_work(512, 512, 39, 16, 32, norm_in_stacks=True)
    norm = a["bm_norm"][1]
    assert norm == 512 * 512 * 2 + 576 * 576 * 8
    # one stack: 2 B in, 256 B out per position, the aggregation sums cleared
    assert a["stack_bior"][1] == 512 * 512 * (2 + 256 + 16)
    # both stage-2 stacks in one launch
    assert a["stack_dct"][1] == 2 * 512 * 512 * (2 + 256) + 512 * 512 * 16
    assert b["stack_bior"][1] == a["stack_bior"][1] + norm
    assert b["stack_dct"][1] == a["stack_dct"][1] + norm


def test_counter_traffic_uses_the_copy_calibration(tmp_path, monkeypatch):
    d = bench.source_digest("reduce")
    f = tmp_path / "traffic.txt"
    f.write_text("# a summary\n"
                 "@copy_fetch_kib_per_byte 0.00048828125\n"
                 "@copy_write_kib_per_byte 0.0009765625\n"
                 f"@kernel_reduce {d} 1000.0 500.0\n"
                 "@kernel_bm 0000000000000000 1.0 1.0\n")
    monkeypatch.setitem(bench.TRAFFIC_FILES, 512, str(f))
    assert bench.measured_traffic("reduce", 512) == pytest.approx(1000.0 / 0.00048828125 + 500.0 / 0.0009765625)
    assert bench.measured_traffic("bm", 512) is None  # taken on other sources
    assert bench.measured_traffic("group_ht", 512) is None  # not in the summary
    monkeypatch.setitem(bench.TRAFFIC_FILES, 512, str(tmp_path / "missing.txt"))
    assert bench.measured_traffic("reduce", 512) is None


def test_instruction_counts_check_the_digest(tmp_path, monkeypatch):
    d = bench.source_digest("bm")
    f = tmp_path / "sq.md"
    f.write_text(f"@sq|bm_corr_kernel<16, 2, 2, false>|{d}|1234.5\n"
                 "@sq|bm_kernel<16, 2, 2, false>|ffffffffffffffff|9\n")
    monkeypatch.setattr(bench, "SQ_FILE", str(f))
    assert bench.measured_valu_insts("bm_corr_kernel<16, 2, 2, false>", "bm") == 1234.5
    assert bench.measured_valu_insts("bm_kernel<16, 2, 2, false>", "bm") is None
    assert bench.measured_valu_insts("bm_corr_kernel<32, 4, 1, false>", "bm") is None


def test_digest_follows_the_sources():
    # every kernel group names sources that exist, and the digest is stable
    for k in bench.KERNEL_SOURCES:
        assert bench.source_digest(k) == bench.source_digest(k)
        assert len(bench.source_digest(k)) == 16


def test_int8_view_counts_64_multiply_accumulates_per_pair():
    v = bench.bm_int8_view(512, 512, 39, 100.0)
    assert v["ops_per_launch"] == 2 * 64 * N512 * (39 * 39 - 1)
    assert v["achieved"] == pytest.approx(v["ops_per_launch"] / 100e-6 / 1e12)
    assert v["frac"] == pytest.approx(v["achieved"] / bench.INT8_MFMA_PEAK_TOPS)


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2", "--no-cpu-baseline"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
