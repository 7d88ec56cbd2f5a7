"""Benchmark: two-stage G-BM3D on one 512 x 512 synthetic image at
sigma = 25/255 on one MI355X, through the C ABI.

A step is one full denoise (block matching, stacks, hard-threshold stage,
pilot quantisation, block matching on the pilot, Wiener stage, aggregation)
of a device-resident uint16 image into a device float image.  Prints one JSON
line.  Per-kernel durations come from HIP events the library records on the
launch stream (a second pass of the same K steps), the roofline entry is for
the kernel with the largest share of the step.
"""
import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0          # MI355X HBM3E
FP64_VALU_PEAK_TFLOPS = 78.6   # 256 CU x 2.4 GHz x 64 lanes x 2 (FMA)
INT8_MFMA_PEAK_TOPS = 5000.0   # dense int8 matrix cores
BF16_MFMA_PEAK_TFLOPS = 2500.0 # dense bf16 matrix cores
# bound -> (peak, unit, scale of the unit)
PEAKS = {"hbm": (HBM_PEAK_GBS, "GB/s", 1e9), "alu": (FP64_VALU_PEAK_TFLOPS, "TFLOP/s", 1e12),
         "mfma": (INT8_MFMA_PEAK_TOPS, "TOP/s", 1e12), "mfma_bf16": (BF16_MFMA_PEAK_TFLOPS, "TFLOP/s", 1e12)}


def algorithmic_work(H, W, search, k1, k2, norm_in_stacks=False):
    """Per-launch algorithmic work of each kernel: bytes for the HBM-bound
    ones; for block matching (either kernel) 5 FLOP of exact arithmetic per
    (pixel, displacement) pair -- one difference, one fused square-accumulate
    (2 FLOP) and the two running-sum additions of the box filter -- on the
    fp64 vector ALU.  norm_in_stacks: the correlation matcher's norm table is
    formed in each stage's stack launch (no norm launch of its own)."""
    from paper_2103_10765_amd import gbm3d
    nref = gbm3d.n_refs(H, W, 3)
    weight_bytes = H * W * 8  # 64-bit block-start weights
    num_bytes = H * W * 8  # 64-bit numerator sums
    S2 = search * search
    norm_bytes = H * W * 2 + (H + 64) * (W + 64) * 8  # pixels in, bordered table out
    in_stack = norm_bytes if norm_in_stacks else 0
    return {
        "bm": ("alu", BM_FLOP_PER_PAIR * H * W * (S2 - 1), "FLOP"),
        # pixels in; one float64 table entry out per bordered position
        "bm_norm": ("hbm", norm_bytes, "B"),
        # the bior launch and the DCT launch (both stage-2 stacks, of the
        # noisy image and of the pilot) clear the weights and numerator sums
        "stack_bior": ("hbm", H * W * (2 + 256) + weight_bytes + num_bytes + in_stack, "B"),
        "stack_dct": ("hbm", 2 * H * W * (2 + 256) + weight_bytes + num_bytes + in_stack, "B"),
        # spectra gathered, ranks read, one 8-byte weight added per block, the
        # image's numerator sums added into once
        "group_ht": ("hbm", nref * (k1 * 256 + 2 * k1 + 8 * k1) + num_bytes, "B"),
        "group_wiener": ("hbm", nref * (2 * k2 * 256 + 2 * k2 + 8 * k2) + num_bytes, "B"),
        "reduce": ("hbm", num_bytes + weight_bytes + H * W * 6, "B"),
    }


BM_FLOP_PER_PAIR = 5


def bm_int8_view(H, W, search, avg_us):
    """The correlation matcher read against the int8 matrix cores instead:
    the 64 multiply-accumulates of one block inner product (2 operations
    each) per (reference, displacement) pair."""
    from paper_2103_10765_amd import gbm3d
    ops = 2.0 * 64 * gbm3d.n_refs(H, W, 3) * (search * search - 1)
    tops = ops / (avg_us * 1e-6) / 1e12
    return {"ops_per_launch": ops, "achieved": tops, "peak": INT8_MFMA_PEAK_TOPS, "unit": "TOP/s",
            "frac": tops / INT8_MFMA_PEAK_TOPS}


TRAFFIC_FILES = {512: os.path.join(ROOT, "profiles", "hbm_traffic_denoise_512.txt"),
                 4096: os.path.join(ROOT, "profiles", "hbm_traffic_denoise_4096.txt")}
KERNEL_SOURCES = {
    "bm": ["bm.hip", "bm_corr.hip", "common.h", "norm.h", "topk.h"], "bm_norm": ["bm_corr.hip", "common.h", "norm.h"],
    "stack_bior": ["stack.hip", "common.h", "norm.h"], "stack_dct": ["stack.hip", "common.h", "norm.h"],
    "group_ht": ["group.hip", "common.h"], "group_wiener": ["group.hip", "common.h"], "reduce": ["group.hip", "common.h"],
}


def source_digest(kernel):
    """sha256 over the sources a kernel is compiled from (first 16 hex digits)."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(ROOT, "paper_2103_10765_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, size=512):
    """HBM bytes per launch of `kernel` on the size x size denoise from the
    committed counter summary: (FETCH_SIZE + WRITE_SIZE) per dispatch, each
    divided by what the same counter reads per byte of a plain device copy of
    known size.  None when the summary is missing or the kernel's sources
    changed since it was taken."""
    path = TRAFFIC_FILES.get(size)
    if not path or not os.path.exists(path):
        return None
    vals = {}
    with open(path) as fh:
        for line in fh:
            parts = line.split()
            if len(parts) >= 2 and parts[0].startswith("@"):
                vals[parts[0][1:]] = parts[1:]
    try:
        fetch_scale = float(vals["copy_fetch_kib_per_byte"][0])
        write_scale = float(vals["copy_write_kib_per_byte"][0])
        digest, fetch_kib, write_kib = vals[f"kernel_{kernel}"][:3]
    except (KeyError, ValueError, IndexError):
        return None
    if digest != source_digest(kernel):
        return None
    return float(fetch_kib) / fetch_scale + float(write_kib) / write_scale


SQ_FILE = os.path.join(ROOT, "profiles", "sq_counters_denoise_512.md")
N_SIMD, CLOCK_HZ = 1024, 2.4e9  # 256 CUs x 4 SIMDs; a wave64 VALU instruction takes 4 SIMD cycles


def measured_valu_insts(variant, kernel):
    """SQ_INSTS_VALU per dispatch of one kernel variant (e.g.
    'bm_corr_kernel<16, 2, 2, false>') from the committed counter summary;
    None when it is missing or the group's sources changed since."""
    if not os.path.exists(SQ_FILE):
        return None
    with open(SQ_FILE) as fh:
        for line in fh:
            parts = line.strip().split("|")
            if len(parts) == 4 and parts[0] == "@sq" and parts[1] == variant:
                return float(parts[3]) if parts[2] == source_digest(kernel) else None
    return None


def copy_calibration(mib):
    """One plain device-to-device copy of `mib` MiB (the reference kernel for
    scaling FETCH_SIZE / WRITE_SIZE to bytes)."""
    import torch
    n = mib << 20
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.zeros(n, dtype=torch.uint8, device="cuda")
    torch.cuda.synchronize()
    y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": n, "ok": bool(y[-1].item() == 1)}), flush=True)


def copy_bandwidth(gib=2, reps=5):
    """Measured HBM bandwidth: a device-to-device copy of `gib` GiB (far past
    the 256 MB last-level cache), read + written bytes over event time."""
    import torch
    n = gib << 30
    x = torch.ones(n, dtype=torch.uint8, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2.0 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del x, y
    torch.cuda.empty_cache()
    return {"copy_GBps": gbps, "bytes": 2 * n}


def unit_peaks(ctx, reps=5):
    """Measured ceilings of the arithmetic units the kernels are read against:
    the library's peak-rate probes (fp64 vector FMA, int8 and bf16 matrix
    cores), 2048 workgroups of 256 threads with no memory traffic."""
    import torch
    from paper_2103_10765_amd import gbm3d
    res = {}
    for name, kind, iters in (("fp64_fma_TFLOPs", gbm3d.PROBE_FP64, 4096),
                              ("int8_mfma_TOPs", gbm3d.PROBE_MFMA_I8, 1024),
                              ("bf16_mfma_TFLOPs", gbm3d.PROBE_MFMA_BF16, 1024)):
        sink, ops = ctx.probe(kind, 2048, iters)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            ctx.probe(kind, 2048, iters, sink=sink)
        e1.record()
        torch.cuda.synchronize()
        res[name] = ops * reps / (e0.elapsed_time(e1) * 1e-3) / 1e12
    return res


def pilot_mfma_executed(n, H, W):
    """Matrix-core FLOP the fused inference kernel issues per batch: 16 x 32
    output tiles, layer l evaluated on the tile grown by 5 - l pixels per side
    in 16-pixel blocks, 2 products per block for layer 0 (its 9 taps x 2
    channels packed into K = 32), 18 for layers 1..4 (9 taps x two 16-channel
    halves), 9 for layer 5 (one half); 16 x 16 x 32 x 2 FLOP each."""
    tiles = n * (-(-H // 16)) * (-(-W // 32))
    blocks = [-(-((16 + 2 * (5 - l)) * (32 + 2 * (5 - l))) // 16) for l in range(6)]
    per_block = [2, 18, 18, 18, 18, 9]
    return tiles * sum(b * m for b, m in zip(blocks, per_block)) * 16 * 16 * 32 * 2


def pilot_conv_rate(ctx, n=32, size=512):
    """Matrix-core rate of the pilot network's inference (all six layers in one
    fused launch) on the evaluation batch shape, from the library-recorded
    events around the launch: the network's own FLOP (`achieved_TFLOPs`) and
    what the kernel issues with the tiles' halos and padding
    (`executed_TFLOPs`)."""
    import numpy as np
    import torch
    from paper_2103_10765_amd import pilot
    rng = np.random.default_rng(7)
    Zt = torch.from_numpy(rng.integers(0, 65536, size=(n, size, size), dtype=np.uint16)).cuda()
    sig = torch.full((n,), 25.0 / 255.0, dtype=torch.float32, device="cuda")
    ctx.pilot_infer(Zt, sig)
    torch.cuda.synchronize()
    ctx.timing(True)
    ctx.timing_reset()
    reps = 3
    for _ in range(reps):
        ctx.pilot_infer(Zt, sig)
    torch.cuda.synchronize()
    tot, launches = ctx.timing_read("pilot_fused")
    ctx.timing(False)
    flop_px = sum(2 * 9 * ci * co for ci, co in pilot.LAYERS)
    tflops = n * size * size * flop_px * reps / (tot * 1e-3) / 1e12
    executed = pilot_mfma_executed(n, size, size)
    return {"conv_ms_per_batch": tot / reps, "launches_per_batch": launches / reps, "flop_per_pixel": flop_px,
            "achieved_TFLOPs": tflops, "peak_TFLOPs": PEAKS["mfma_bf16"][0], "frac": tflops / PEAKS["mfma_bf16"][0],
            "executed_flop_per_batch": executed, "executed_TFLOPs": executed * reps / (tot * 1e-3) / 1e12}


def sigma_bench(ctx, p, Zt_shape, steps=50):
    """The 512^2 image at sigma 15, 25 and 50 / 255: Mpixel/s and PSNR."""
    import numpy as np
    import torch
    from paper_2103_10765_amd.gbm3d import psnr_db
    from paper_2103_10765_amd import synth
    H, W = Zt_shape
    res = {}
    for s255 in (15.0, 25.0, 50.0):
        sigma = s255 / 255.0
        clean, Z = synth.make_case(H, W, sigma, 2)
        Zt = torch.from_numpy(Z).cuda()
        out = torch.empty((H, W), dtype=torch.float32, device="cuda")
        for _ in range(3):
            ctx.denoise(Zt, sigma, p, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.denoise(Zt, sigma, p, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[f"{s255:g}"] = {"mpix_s": H * W / (ms * 1e-3) / 1e6,
                            "psnr_db": psnr_db(out.cpu().numpy().astype(np.float64), clean),
                            "psnr_noisy_db": psnr_db(Z / 65535.0, clean)}
    return res


def global_bench(ctx, Zt, clean, sigma, steps=20):
    """The volume form of stage 1 (tiles of 16, one 3-D transform of the
    whole volume, 2 cycle spins, 2 translations) against the grouped stage 1
    on the same image: Mpixel/s and PSNR of each."""
    import numpy as np
    import torch
    from paper_2103_10765_amd.gbm3d import psnr_db
    H, W = Zt.shape
    out = torch.empty((H, W), dtype=torch.float32, device="cuda")

    def timed(fn, n=steps):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(n):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / n

    from paper_2103_10765_amd import gbm3d
    gp = gbm3d.global_default_params()
    ms_g = timed(lambda: ctx.global_basic(Zt, sigma, out=out))
    p_g = psnr_db(out.cpu().numpy().astype(np.float64), clean)
    ms_b = timed(lambda: ctx.basic(Zt, sigma, out=out))
    p_b = psnr_db(out.cpu().numpy().astype(np.float64), clean)
    # its largest kernel, the tile matching, alone through its own entry
    # point (one translation per launch; inside the stage all translations
    # share one launch): exact distances, 3 FLOP per (pixel, displacement)
    # as for the grouped matcher, on the fp64 vector ALU
    ms_m = timed(lambda: ctx.global_match(Zt, gp))
    flop = 3.0 * H * W * (gp.search * gp.search - 1)
    tflops = flop / (ms_m * 1e-3) / 1e12
    mpx = H * W / 1e6
    # the 4096^2 edge-rich image, volume form only
    from paper_2103_10765_amd import synth
    _, Zl = synth.large_image_case(4096, sigma, 4)
    Zlt = torch.from_numpy(Zl).cuda()
    outl = torch.empty(Zlt.shape, dtype=torch.float32, device="cuda")
    ms_l = timed(lambda: ctx.global_basic(Zlt, sigma, out=outl), n=3)
    del Zlt, outl
    torch.cuda.empty_cache()
    return {"global_ms": ms_g, "global_mpix_s": mpx / (ms_g * 1e-3), "global_psnr_db": p_g,
            "grouped_ms": ms_b, "grouped_mpix_s": mpx / (ms_b * 1e-3), "grouped_psnr_db": p_b,
            "global_4096_ms": ms_l, "global_4096_mpix_s": 4096 * 4096 / 1e6 / (ms_l * 1e-3),
            # context from another machine: the paper's stage 1 in this volume
            # form (Table 2, MATLAB with GPU filtering and CPU matching)
            "paper_table2_g_bm3d1_s": {"512": 0.334, "4096": 14.08},
            "roofline": {"kernel": "gl_match_kernel", "bound": "alu", "avg_us": 1e3 * ms_m,
                         "translations_per_call": gp.n_shifts, "work_per_launch": flop, "work_unit": "FLOP",
                         "achieved": tflops, "peak": FP64_VALU_PEAK_TFLOPS, "unit": "TFLOP/s",
                         "frac": tflops / FP64_VALU_PEAK_TFLOPS}}


def tiled_bench(ctx, sigma, steps=5):
    """The two-stage denoise on 256 + 8 sub-images (stride 256, both stages
    of all sub-images in one batched call each) beside the whole-image call,
    at 512^2 and on the 4096^2 edge-rich image: ms, Mpixel/s and PSNR."""
    import numpy as np
    import torch
    from paper_2103_10765_amd import synth, tiled
    from paper_2103_10765_amd.gbm3d import psnr_db
    res = {"size": tiled.SIZE, "stride": tiled.STRIDE}
    for name, (clean, Z) in (("512", synth.make_case(512, 512, sigma, 2)),
                             ("4096", synth.large_image_case(4096, sigma, 4))):
        Zt = torch.from_numpy(Z).cuda()
        row = {}
        for mode, fn in (("tiled", lambda: tiled.denoise(ctx, Zt, sigma)[0]), ("whole", lambda: ctx.denoise(Zt, sigma))):
            out = fn()
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                out = fn()
            e1.record()
            torch.cuda.synchronize()
            ms = e0.elapsed_time(e1) / steps
            row[mode] = {"ms": ms, "mpix_s": Z.size / (ms * 1e-3) / 1e6,
                         "psnr_db": psnr_db(out.cpu().numpy().astype(np.float64), clean)}
        res[name] = row
        del Zt
        torch.cuda.empty_cache()
    return res


def recompute_bench(ctx, sigma, steps=10):
    """Stage 1 with every block's bior1.5 spectrum read from the precomputed
    stack (default) against computed inside the group kernel from the block's
    pixels (no stack), at 512^2 and on the 4096^2 edge-rich image: ms per
    stage-1 call (matching included) and of the group kernel alone."""
    import torch
    from paper_2103_10765_amd import gbm3d, synth
    res = {}
    for name, (_, Z) in (("512", synth.make_case(512, 512, sigma, 2)),
                         ("4096", synth.large_image_case(4096, sigma, 4))):
        Zt = torch.from_numpy(Z).cuda()
        out = torch.empty(Zt.shape, dtype=torch.float32, device="cuda")
        row = {}
        for mode, src in (("stack", gbm3d.HT_STACK), ("recompute", gbm3d.HT_RECOMPUTE)):
            p = gbm3d.default_params(ht_source=src)
            ctx.basic(Zt, sigma, p, out=out)
            torch.cuda.synchronize()
            e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            e0.record()
            for _ in range(steps):
                ctx.basic(Zt, sigma, p, out=out)
            e1.record()
            torch.cuda.synchronize()
            ctx.timing(True)
            ctx.timing_reset()
            ctx.basic(Zt, sigma, p, out=out)
            torch.cuda.synchronize()
            tot, n = ctx.timing_read("group_ht")
            ctx.timing(False)
            row[mode] = {"stage1_ms": e0.elapsed_time(e1) / steps, "group_ht_ms": tot / max(n, 1)}
        res[name] = row
        del Zt, out
        torch.cuda.empty_cache()
    return res


def cpu_baseline(Z, sigma, size=320):
    """The CPU oracle (one thread) on a size x size crop of the same image."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import gbm3d_oracle as O
    crop = np.ascontiguousarray(Z[:size, :size])
    with threadpool_limits(limits=1):
        t0 = time.perf_counter()
        O.denoise(crop, sigma)
        dt = time.perf_counter() - t0
    return {"value": size * size / dt / 1e6, "unit": "Mpixel/s", "cores": 1, "kind": "oracle",
            "sample": f"two-stage denoise of the top-left {size}x{size} crop of the benchmark image, "
                      f"{dt:.1f} s, float64 NumPy, 1 thread"}


def host_cpu():
    """The host's CPU model (first 'model name' of /proc/cpuinfo)."""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def _oracle_crop(spec):
    """Worker of cpu_pool_baseline: the oracle on one crop of a batch image."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import gbm3d_oracle as O
    from paper_2103_10765_amd import synth
    h, w, s, sd, size = spec
    _, Z = synth.make_case(h, w, s, sd)
    with threadpool_limits(limits=1):
        O.denoise(np.ascontiguousarray(Z[:size, :size]), s)
    return size * size


def cpu_pool_baseline(size=128, rounds=2):
    """The CPU oracle over the uneven batch's images (top-left size x size
    crop of each, its own sigma) in a process pool of every usable host core
    (at most 16), one thread per process; Mpixel/s over the whole pool."""
    import multiprocessing as mp
    from paper_2103_10765_amd import synth
    cores = max(1, min(16, len(os.sched_getaffinity(0))))
    specs = [(h, w, s, sd, size) for (h, w, s, sd) in synth.batch_specs()][:cores * rounds]
    with mp.get_context("spawn").Pool(cores) as pool:
        pool.map(_oracle_crop, specs[:cores])  # start-up and imports outside the timed part
        t0 = time.perf_counter()
        px = sum(pool.map(_oracle_crop, specs))
        dt = time.perf_counter() - t0
    return {"value": px / dt / 1e6, "unit": "Mpixel/s", "cores": cores, "kind": "oracle",
            "sample": f"two-stage denoise of the top-left {size}x{size} crops of the first {len(specs)} images "
                      f"of the 64-image batch (each at its own sigma), {dt:.1f} s, one process per core"}


def batch_bench(ctx, reps=5):
    """64 images of uneven sizes (256..1024 per side), sigma U[10,50]/255, one
    batched call under hipGraph replay; Mpixel/s over all images."""
    import torch
    from paper_2103_10765_amd import synth
    specs = synth.batch_specs()
    imgs, sig = [], []
    for (h, w, s, sd) in specs:
        _, Z = synth.make_case(h, w, s, sd)
        imgs.append(torch.from_numpy(Z).cuda())
        sig.append(s)
    outs = [torch.empty(tuple(x.shape), dtype=torch.float32, device="cuda") for x in imgs]
    ctx.denoise_batch(imgs, sig, outs=outs, graph=True)   # capture
    torch.cuda.synchronize()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        ctx.denoise_batch(imgs, sig, outs=outs, graph=True)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    mpx = sum(h * w for (h, w, _, _) in specs) / 1e6
    return {"images": len(specs), "mpixels": mpx, "ms_per_batch": ms, "mpix_s": mpx / (ms * 1e-3),
            "mode": "hipGraph replay, one workgroup per work item of the whole batch"}


def size_bench(ctx, p):
    """Two-stage Mpixel/s on the small (128^2, seed 1) and the large
    (4096^2 with edge-rich rectangles, seed 4) single images, sigma 25/255."""
    import torch
    from paper_2103_10765_amd import synth
    res = {}
    for name, (clean, Z), steps in (("128x128", synth.make_case(128, 128, synth.SIGMA25, 1), 50),
                                     ("4096x4096", synth.large_image_case(4096, synth.SIGMA25, 4), 3)):
        Zt = torch.from_numpy(Z).cuda()
        out = torch.empty(Zt.shape, dtype=torch.float32, device="cuda")
        ctx.denoise(Zt, synth.SIGMA25, p, out=out)
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(steps):
            ctx.denoise(Zt, synth.SIGMA25, p, out=out)
        e1.record()
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[name] = {"ms_per_image": ms, "mpix_s": Z.size / (ms * 1e-3) / 1e6, "steps": steps}
        del Zt, out
        torch.cuda.empty_cache()
    return res


def kernels_4096(ctx, p, steps=3):
    """Per-kernel entries (as for the benchmark image) on the 4096^2
    edge-rich image at sigma 25/255, where the patch stacks (4.3 GB each) are
    far larger than the 256 MB last-level cache: the HBM-bound kernels' true
    test."""
    import torch
    from paper_2103_10765_amd import synth
    _, Z = synth.large_image_case(4096, synth.SIGMA25, 4)
    Zt = torch.from_numpy(Z).cuda()
    ctx.denoise(Zt, synth.SIGMA25, p)
    torch.cuda.synchronize()
    res = per_kernel(ctx, Zt, synth.SIGMA25, p, steps)
    del Zt
    torch.cuda.empty_cache()
    return res


def pilot_bench(ctx):
    """Learned pilot vs plain stage 1, both followed by the Wiener stage, on the
    32 x 512^2 evaluation batch at sigma 25/255 (needs trained weights)."""
    import numpy as np
    import torch
    from paper_2103_10765_amd import pilot
    if not os.path.exists(pilot.DEFAULT_WEIGHTS):
        return {"skipped": "no trained pilot weights (python -m paper_2103_10765_amd.pilot train)"}
    with np.load(pilot.DEFAULT_WEIGHTS, allow_pickle=False) as f:
        master = torch.from_numpy(f["master"]).cuda()
    return pilot.evaluate(ctx, master, log=lambda s: None)


def per_kernel(ctx, Zt, sigma, p, steps, variants=None):
    """Average duration per launch of every kernel of the two-stage denoise
    of Zt (library-recorded HIP events on the launch stream around each
    launch, over `steps` denoise calls), with its algorithmic work against
    the unit's spec peak, the counter-measured HBM bytes of the committed
    summary for this image size (when the kernel's sources have not changed
    since), and, with `variants`, the vector-instruction issue fraction."""
    import torch
    H, W = (int(v) for v in Zt.shape)
    ctx.timing(True)
    ctx.timing_reset()
    for _ in range(steps):
        ctx.denoise(Zt, sigma, p)
    torch.cuda.synchronize()
    kernels = {}
    for name in ("bm", "bm_norm", "stack_bior", "stack_dct", "group_ht", "group_wiener", "reduce"):
        tot, n = ctx.timing_read(name)
        if n:
            kernels[name] = {"avg_us": 1e3 * tot / n, "launches_per_step": n / steps, "ms_per_step": tot / steps}
    ctx.timing(False)
    # no norm launch of its own: the stack launches formed the norm tables
    work = algorithmic_work(H, W, p.search, p.k_ht, p.k_wiener,
                            norm_in_stacks="bm_norm" not in kernels and "bm" in kernels)
    for name, k in kernels.items():
        bound, amount, unit = work[name]
        peak, punit, scale = PEAKS[bound]
        k["bound"] = bound
        k["work_per_launch"] = amount
        k["work_unit"] = unit
        # `frac` is algorithmic work over time against the spec peak; what the
        # HBM counters saw is `hbm_counted_frac` (null without a current summary)
        k["work_basis"] = "algorithmic"
        k["achieved"] = amount / (k["avg_us"] * 1e-6) / scale
        k["peak"] = peak
        k["unit"] = punit
        k["frac"] = k["achieved"] / peak
        tb = measured_traffic(name, H if H == W else 0)
        k["traffic_bytes"] = tb
        if tb is not None:
            # what the counters saw leave and enter HBM, over the same time
            k["hbm_counted_GBps"] = tb / (k["avg_us"] * 1e-6) / 1e9
            k["hbm_counted_frac"] = k["hbm_counted_GBps"] / HBM_PEAK_GBS
        if name == "bm":
            k["int8_view"] = bm_int8_view(H, W, p.search, k["avg_us"])
        if variants:
            # vector-instruction issue: committed SQ_INSTS_VALU of the same
            # variants x 4 cycles over every SIMD's cycles of the measured time
            insts = [measured_valu_insts(v, name) if v else None for v in variants.get(name, [])]
            if insts and None not in insts:
                k["valu_issue_frac"] = sum(insts) * 4 / (N_SIMD * CLOCK_HZ * len(insts) * k["avg_us"] * 1e-6)
    return kernels


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--size", type=int, default=512)
    ap.add_argument("--sigma", type=float, default=25.0)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-extras", action="store_true", help="skip the batch and learned-pilot measurements")
    ap.add_argument("--bm-method", choices=["tuned", "shift", "corr"], default="tuned",
                    help="block-matching kernel: autotuned on the benchmark image (default) or fixed")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run one plain device copy of MIB MiB (counter calibration) and exit")
    ap.add_argument("--batch-only", action="store_true",
                    help="only time the 64-image batch under graph replay (for profiling the batch path)")
    ap.add_argument("--global-only", action="store_true",
                    help="only time the volume form of stage 1 beside the grouped stage 1 (for profiling it)")
    ap.add_argument("--pilot-only", action="store_true",
                    help="only time the learned pilot's fused inference on 32 x 512^2 (for profiling it)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration(args.copy_calibration)
        return
    if args.batch_only:
        from paper_2103_10765_amd import gbm3d
        ctx = gbm3d.Context(0)
        print(json.dumps(batch_bench(ctx, reps=args.steps)), flush=True)
        ctx.close()
        return
    if args.pilot_only:
        import numpy as np
        import torch
        from paper_2103_10765_amd import gbm3d, pilot
        ctx = gbm3d.Context(0)
        with np.load(pilot.DEFAULT_WEIGHTS, allow_pickle=False) as f:
            ctx.pilot_load(torch.from_numpy(f["master"]).cuda())
        print(json.dumps(pilot_conv_rate(ctx)), flush=True)
        ctx.close()
        return
    if args.global_only:
        import torch
        from paper_2103_10765_amd import gbm3d, synth
        sigma = args.sigma / 255.0
        clean, Z = synth.make_case(args.size, args.size, sigma, 2)
        ctx = gbm3d.Context(0)
        print(json.dumps(global_bench(ctx, torch.from_numpy(Z).cuda(), clean, sigma, steps=args.steps)), flush=True)
        ctx.close()
        return
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (asked for --gpus {args.gpus}); "
              "images are independent, so a multi-GPU run is a per-GPU split of the batch", file=sys.stderr)
        sys.exit(2)

    # the multi-core oracle baseline first: its worker processes start before
    # this process touches the GPU
    pool_baseline = None
    if not args.no_cpu_baseline and not args.no_extras:
        pool_baseline = cpu_pool_baseline()

    import numpy as np
    import torch

    from paper_2103_10765_amd.gbm3d import psnr_db
    from paper_2103_10765_amd import gbm3d, synth

    sigma = args.sigma / 255.0
    H = W = args.size
    clean, Z = synth.make_case(H, W, sigma, 2)
    dev = torch.device("cuda:0")
    Zt = torch.from_numpy(Z).to(dev)
    out = torch.empty((H, W), dtype=torch.float32, device=dev)
    ctx = gbm3d.Context(0)
    p = gbm3d.default_params()
    stream = torch.cuda.current_stream()
    tuned = {}
    if args.bm_method == "tuned":
        # stage 2 matches on the pilot; the noisy image has the same shape class
        for K in (p.k_ht, p.k_wiener):
            m, sp, t = ctx.autotune(Zt, K, reps=3)
            tuned[f"K{K}"] = {"method": {1: "shift", 2: "corr"}[m], "split": sp, "ms": t}
        # the stage-1 group-kernel shape the autotuner chose (from its records)
        import tempfile
        with tempfile.TemporaryDirectory() as td:
            ctx.tune_save(os.path.join(td, "tune.txt"))
            for ln in open(os.path.join(td, "tune.txt")):
                f = ln.split()
                if f[0] == "ht" and int(f[1]) == p.k_ht and int(f[2]) == p.search:
                    tuned["stage1_groups"] = {"shape": ["two tiles of 12 waves per CU",
                                                        "one tile of 16 waves, prefetch"][int(f[4])],
                                              "ms_stage1": float(f[5])}
    else:
        p.bm_method = {"shift": gbm3d.BM_SHIFT, "corr": gbm3d.BM_CORR}[args.bm_method]

    for _ in range(args.warmup):
        ctx.denoise(Zt, sigma, p, out=out)
    torch.cuda.synchronize()

    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    t0 = time.perf_counter()
    e0.record(stream)
    for _ in range(args.steps):
        ctx.denoise(Zt, sigma, p, out=out)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1) / args.steps
    value = H * W / (ms * 1e-3) / 1e6

    Y = out.cpu().numpy().astype(np.float64)
    psnr = psnr_db(Y, clean)

    # per-kernel durations: the same steps with library-recorded events
    # the kernel variants this run launched, for the instruction counters
    def bm_variant(K):
        t = tuned.get(f"K{K}")
        if not t:
            return None
        s = t["split"]
        return f"{'bm_corr_kernel' if t['method'] == 'corr' else 'bm_kernel'}<{K}, {4 // s}, {s}, false>"
    def stack_variant(K, kind):
        # the stack launch carries the norm table when the correlation kernel
        # matches; the 512^2 launches are short ones (pixel loads all at once)
        t = tuned.get(f"K{K}")
        return f"stack_norm_kernel<{kind}, true>" if t and t["method"] == "corr" else f"stack_kernel<{kind}, false>"
    variants = {"bm": [bm_variant(p.k_ht), bm_variant(p.k_wiener)], "bm_norm": ["bm_norm_kernel<false>"] * 2,
                "stack_bior": [stack_variant(p.k_ht, 0)], "stack_dct": [stack_variant(p.k_wiener, 1)],
                "group_ht": [f"group_ht_kernel<{p.k_ht}, false, false, "
                             f"{'false' if tuned.get('stage1_groups', {}).get('shape', '').startswith('one') else 'true'}>"],
                "group_wiener": [f"group_wiener_kernel<{p.k_wiener}, false>"], "reduce": ["reduce_kernel<false>"] * 2}
    # (the committed instruction counts are those of the 512^2 image)
    kernels = per_kernel(ctx, Zt, sigma, p, args.steps, variants if H == W == 512 else None)
    dom = max(kernels, key=lambda n: kernels[n]["ms_per_step"])
    k = kernels[dom]
    roof = {"bound": k["bound"], "kernel": dom, "achieved": k["achieved"], "peak": k["peak"], "unit": k["unit"],
            "frac": k["frac"], "traffic": k["traffic_bytes"], "avg_us": k["avg_us"],
            "work_per_launch": k["work_per_launch"], "work_unit": k["work_unit"],
            "valu_issue_frac": k.get("valu_issue_frac")}
    if "int8_view" in k:
        roof["int8_view"] = k["int8_view"]

    rec = {
        "metric": "Mpixel/s two-stage denoise at sigma=25 (plain vs learned pilot) + PSNR gap, 1 GPU",
        "value": value,
        "unit": "Mpixel/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms,
        "wall_s": wall,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"plain G-BM3D two-stage, one {H}x{W} grayscale image, sigma={args.sigma:g}/255, "
                               "patch 8, step 3, search 39, K 16/32", "image_seed": 2,
                   "block_matching": tuned if tuned else args.bm_method},
        "psnr_db": psnr,
        "psnr_noisy_db": psnr_db(Z / 65535.0, clean),
        "psnr_gap_db": None,
        "roofline": roof,
        "kernels": kernels,
    }
    if not args.no_extras:
        pb = pilot_bench(ctx)
        rec["pilot"] = pb
        if "psnr_gap_db" in pb:
            rec["psnr_gap_db"] = pb["psnr_gap_db"]
        if "skipped" not in pb:
            rec["pilot"]["conv"] = pilot_conv_rate(ctx)
        rec["batch"] = batch_bench(ctx)
        rec["sizes"] = size_bench(ctx, p)
        rec["kernels_4096"] = kernels_4096(ctx, p)
        rec["sigmas"] = sigma_bench(ctx, p, (H, W))
        from paper_2103_10765_amd import pnp
        rec["pnp"] = pnp.bench(ctx)
        rec["global_stage1"] = global_bench(ctx, Zt, clean, sigma)
        rec["tiled_sub_images"] = tiled_bench(ctx, sigma)
        rec["stage1_recompute"] = recompute_bench(ctx, sigma)
        mp = copy_bandwidth()
        mp.update(unit_peaks(ctx))
        rec["measured_peaks"] = mp
        measured = {"hbm": mp["copy_GBps"], "alu": mp["fp64_fma_TFLOPs"], "mfma": mp["int8_mfma_TOPs"]}
        for k in kernels.values():
            if k["bound"] == "hbm":
                k["frac_of_measured_copy"] = k["achieved"] / mp["copy_GBps"]
            k["frac_of_measured_peak"] = k["achieved"] / measured[k["bound"]]
        for k in rec["kernels_4096"].values():
            if k["bound"] == "hbm":
                k["frac_of_measured_copy"] = k["achieved"] / mp["copy_GBps"]
                if "hbm_counted_GBps" in k:
                    k["hbm_counted_frac_of_copy"] = k["hbm_counted_GBps"] / mp["copy_GBps"]
            k["frac_of_measured_peak"] = k["achieved"] / measured[k["bound"]]
        for k in kernels.values():
            if "hbm_counted_GBps" in k:
                k["hbm_counted_frac_of_copy"] = k["hbm_counted_GBps"] / mp["copy_GBps"]
        roof["frac_of_measured_peak"] = roof["achieved"] / measured[roof["bound"]]
        gr = rec["global_stage1"]["roofline"]
        gr["frac_of_measured_peak"] = gr["achieved"] / mp["fp64_fma_TFLOPs"]
        if "conv" in rec.get("pilot", {}):
            c = rec["pilot"]["conv"]
            c["frac_of_measured_peak"] = c["achieved_TFLOPs"] / mp["bf16_mfma_TFLOPs"]
    if not args.no_cpu_baseline:
        rec["cpu_baseline"] = cpu_baseline(Z, sigma)
        rec["cpu_baseline"]["host_cpu"] = host_cpu()
        if pool_baseline is not None:
            rec["cpu_baseline_pool"] = pool_baseline
    print(json.dumps(rec), flush=True)
    ctx.close()


if __name__ == "__main__":
    main()
