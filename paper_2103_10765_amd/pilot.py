"""Learned pilot: training and evaluation drivers.

The network and its kernels live in the library (gbm3d_pilot_*); this module
generates the training pairs (noisy crop, G-BM3D basic estimate of it, both
produced with the library's own batched stage 1), runs Adam with a cosine
learning-rate schedule through the library's gradient and update kernels,
writes and resumes checkpoints (NumPy .npz, no pickled objects), and compares
learned-pilot two-stage denoising with the plain two-stage path.

    python -m paper_2103_10765_amd.pilot train --crops 20000 --steps 200000 --weighting sigma --out w.npz
    python -m paper_2103_10765_amd.pilot eval --weights w.npz
"""
from __future__ import annotations

import argparse
import concurrent.futures as cf
import json
import os
import sys
import time

import numpy as np

from . import synth

LAYERS = [(2, 32), (32, 32), (32, 32), (32, 32), (32, 32), (32, 1)]
N_PARAMS = sum(9 * ci * co + co for ci, co in LAYERS)
DEFAULT_WEIGHTS = os.path.join(os.path.dirname(os.path.abspath(__file__)), "pilot_weights.npz")


def init_params(seed: int = 0) -> np.ndarray:
    """He-normal weights (std sqrt(2 / fan_in)) in W[ky][kx][ci][co] order,
    zero biases; the last layer is scaled by 0.1 so the first pilots stay close
    to the noisy image."""
    rng = np.random.default_rng(seed)
    parts = []
    for l, (ci, co) in enumerate(LAYERS):
        W = rng.standard_normal(9 * ci * co) * np.sqrt(2.0 / (9 * ci))
        if l == len(LAYERS) - 1:
            W *= 0.1
        parts += [W, np.zeros(co)]
    out = np.concatenate(parts).astype(np.float32)
    assert out.size == N_PARAMS
    return out


def _crop(args):
    i, sigma, size = args
    _, Z = synth.pilot_train_crop(i, sigma, size)
    return Z


def make_crops(n: int, size: int = 128, workers: int = 8):
    """n seeded noisy crops (uint16 [n, size, size]) and their sigmas."""
    sig = synth.pilot_train_sigmas(max(n, 1))[:n].astype(np.float32)
    jobs = [(i, float(sig[i]), size) for i in range(n)]
    if workers > 1 and n > 64:
        with cf.ProcessPoolExecutor(max_workers=workers) as ex:
            Z = list(ex.map(_crop, jobs, chunksize=64))
    else:
        Z = [_crop(j) for j in jobs]
    return np.stack(Z), sig


def basic_targets(ctx, Zt, sig, chunk: int = 512):
    """Stage-1 estimates of every crop (device float [n, H, W]) via the batch API."""
    import torch
    n = Zt.shape[0]
    out = torch.empty(Zt.shape, dtype=torch.float32, device=Zt.device)
    for s in range(0, n, chunk):
        e = min(n, s + chunk)
        imgs = [Zt[i] for i in range(s, e)]
        outs = [out[i] for i in range(s, e)]
        ctx.denoise_batch(imgs, [float(x) for x in sig[s:e]], outs=outs, basic_only=True)
    torch.cuda.synchronize()
    return out


def save_checkpoint(path, master, m, v, step, meta=None):
    tmp = path + ".tmp.npz"
    np.savez(tmp, master=master.cpu().numpy(), m=m.cpu().numpy(), v=v.cpu().numpy(),
             step=np.array([step], dtype=np.int64), meta=np.frombuffer(json.dumps(meta or {}).encode(), np.uint8))
    os.replace(tmp, path)


def load_checkpoint(path):
    with np.load(path, allow_pickle=False) as f:
        meta = json.loads(bytes(f["meta"]).decode()) if "meta" in f else {}
        return f["master"], f["m"], f["v"], int(f["step"][0]), meta


def lr_at(step: int, total: int, lr0: float = 1e-3, lr1: float = 1e-5) -> float:
    """Cosine decay from lr0 to lr1 over `total` steps."""
    t = min(max(step - 1, 0) / max(total - 1, 1), 1.0)
    return lr1 + 0.5 * (lr0 - lr1) * (1.0 + np.cos(np.pi * t))


def loss_weights(sig_t, mode: str):
    """Per-crop loss weights: 'none' (plain mean squared error) or 'sigma'
    ((sigma_ref / sigma)^2 with sigma_ref = 25/255, so that every noise level
    contributes errors of the same relative size)."""
    if mode == "none":
        return None
    if mode == "sigma":
        return (synth.SIGMA25 / sig_t) ** 2
    raise ValueError(mode)


def train(ctx, Zt, target, sig_t, steps: int, batch: int = 64, seed: int = 0, ckpt: str | None = None,
          ckpt_every: int = 500, resume: bool = True, log=print, weighting: str = "none", hist_every: int = 100,
          stop_after: int | None = None):
    """Adam on the (optionally per-crop weighted) mean squared error between
    the pilot and the stage-1 target.  The batch order is a seeded permutation
    per epoch, so a resumed run continues exactly where it stopped.  The loss
    is recorded every `hist_every` steps; `stop_after` ends the run after that
    step (checkpointed when `ckpt` is set), as an interrupted run would."""
    import torch
    n = Zt.shape[0]
    dev = Zt.device
    step0 = 0
    if ckpt and resume and os.path.exists(ckpt):
        w, m, v, step0, _ = load_checkpoint(ckpt)
        master, m, v = (torch.from_numpy(a).to(dev) for a in (w, m, v))
        log(f"resumed from {ckpt} at step {step0}")
    else:
        master = torch.from_numpy(init_params(seed)).to(dev)
        m = torch.zeros_like(master)
        v = torch.zeros_like(master)
    ctx.pilot_load(master)
    grad = torch.empty_like(master)
    loss = torch.empty(1, dtype=torch.float32, device=dev)
    per_epoch = max(n // batch, 1)
    w_all = loss_weights(sig_t, weighting)
    t0 = time.perf_counter()
    hist = []
    for step in range(step0 + 1, steps + 1):
        epoch, k = divmod(step - 1, per_epoch)
        perm = np.random.default_rng(seed * 100003 + epoch).permutation(n)
        ids = torch.from_numpy(perm[k * batch:(k + 1) * batch].astype(np.int64)).to(dev)
        ctx.pilot_grad(Zt.index_select(0, ids).contiguous(), target.index_select(0, ids).contiguous(),
                       sig_t.index_select(0, ids).contiguous(), grad=grad, loss=loss,
                       weight=None if w_all is None else w_all.index_select(0, ids).contiguous())
        ctx.pilot_adam(master, m, v, grad, step, lr_at(step, steps))
        if step % hist_every == 0 or step == steps:
            hist.append((step, loss.item()))
            log(f"step {step} loss {hist[-1][1]:.3e} lr {lr_at(step, steps):.2e} {time.perf_counter() - t0:.1f}s")
        stop = stop_after is not None and step >= stop_after
        if ckpt and (step % ckpt_every == 0 or step == steps or stop):
            save_checkpoint(ckpt, master, m, v, step, {"batch": batch, "seed": seed, "steps": steps,
                                                       "weighting": weighting})
        if stop:
            break
    torch.cuda.synchronize()
    return master, hist


def evaluate(ctx, master, n: int = 32, size: int = 512, sigma: float = synth.SIGMA25, reps: int = 5, log=print):
    """Learned-pilot vs plain two-stage denoising of n size x size images:
    Mpixel/s of each (device-resident inputs, batched, graph replay) and the
    mean PSNR of each against the clean images."""
    import torch
    from .gbm3d import psnr_db
    cases = synth.pilot_eval_cases(n, size, sigma)
    dev = torch.device("cuda", ctx.device)
    Zt = torch.from_numpy(np.stack([Z for _, Z in cases])).to(dev)
    imgs = [Zt[i] for i in range(n)]
    sig = [float(sigma)] * n
    sig_t = torch.full((n,), float(sigma), dtype=torch.float32, device=dev)
    ctx.pilot_load(master)
    out_plain = [torch.empty((size, size), dtype=torch.float32, device=dev) for _ in range(n)]
    out_learn = [torch.empty((size, size), dtype=torch.float32, device=dev) for _ in range(n)]

    def plain():
        ctx.denoise_batch(imgs, sig, outs=out_plain, graph=True)

    def learned():
        pu, _ = ctx.pilot_infer(Zt, sig_t)
        ctx.denoise_batch(imgs, sig, pilots=[pu[i] for i in range(n)], outs=out_learn, graph=True)

    def timed(fn):
        fn()
        torch.cuda.synchronize()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        e0.record()
        for _ in range(reps):
            fn()
        e1.record()
        torch.cuda.synchronize()
        return e0.elapsed_time(e1) / reps

    ms_plain = timed(plain)
    ms_learn = timed(learned)
    clean = [c for c, _ in cases]
    p_plain = float(np.mean([psnr_db(o.cpu().numpy(), c) for o, c in zip(out_plain, clean)]))
    p_learn = float(np.mean([psnr_db(o.cpu().numpy(), c) for o, c in zip(out_learn, clean)]))
    mpx = n * size * size / 1e6
    res = {"images": n, "size": size, "sigma_255": sigma * 255,
           "plain_ms": ms_plain, "learned_ms": ms_learn,
           "plain_mpix_s": mpx / (ms_plain * 1e-3), "learned_mpix_s": mpx / (ms_learn * 1e-3),
           "plain_psnr_db": p_plain, "learned_psnr_db": p_learn, "psnr_gap_db": p_plain - p_learn}
    log(json.dumps(res))
    return res


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("train")
    t.add_argument("--crops", type=int, default=20000)
    t.add_argument("--size", type=int, default=128)
    t.add_argument("--steps", type=int, default=200000)
    t.add_argument("--batch", type=int, default=64)
    t.add_argument("--seed", type=int, default=0)
    t.add_argument("--out", default=DEFAULT_WEIGHTS)
    t.add_argument("--ckpt", default=None)
    t.add_argument("--workers", type=int, default=8)
    t.add_argument("--eval", action="store_true")
    t.add_argument("--weighting", choices=["none", "sigma"], default="sigma")
    e = sub.add_parser("eval")
    e.add_argument("--weights", default=DEFAULT_WEIGHTS)
    e.add_argument("--n", type=int, default=32)
    e.add_argument("--size", type=int, default=512)
    args = ap.parse_args(argv)

    import torch
    from . import gbm3d
    ctx = gbm3d.Context(0)
    if args.cmd == "train":
        t0 = time.perf_counter()
        Z, sig = make_crops(args.crops, args.size, args.workers)
        print(f"crops {Z.shape} in {time.perf_counter() - t0:.1f}s", flush=True)
        Zt = torch.from_numpy(Z).cuda()
        sig_t = torch.from_numpy(sig).cuda()
        t1 = time.perf_counter()
        target = basic_targets(ctx, Zt, sig)
        print(f"stage-1 targets in {time.perf_counter() - t1:.1f}s", flush=True)
        master, _ = train(ctx, Zt, target, sig_t, args.steps, args.batch, args.seed, ckpt=args.ckpt,
                          log=lambda s: print(s, flush=True), weighting=args.weighting)
        np.savez(args.out, master=master.cpu().numpy())
        print(f"saved {args.out}", flush=True)
        if args.eval:
            evaluate(ctx, master, log=lambda s: print(s, flush=True))
    else:
        with np.load(args.weights, allow_pickle=False) as f:
            master = torch.from_numpy(f["master"]).cuda()
        evaluate(ctx, master, args.n, args.size, log=lambda s: print(s, flush=True))
    ctx.close()


if __name__ == "__main__":
    main(sys.argv[1:])
