"""ctypes binding of libgbm3d.so (the C ABI in include/gbm3d.h).

Argument marshalling only: every step of the denoiser runs in the library's
HIP kernels.  Tensors supply device memory; the current torch stream is passed
as the HIP stream.  There is no CPU fallback: if the library is missing,
loading raises.
"""
from __future__ import annotations

import ctypes
import os

import torch  # loaded first so the library binds to the same HIP runtime as torch

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libgbm3d.so")

OK, EINVAL, EUNSUPPORTED, ENOMEM, EHIP = 0, -1, -2, -3, -4
BATCH_GRAPH, BATCH_BASIC_ONLY = 1, 2
W_TV, W_NNZ, W_UNIT = 0, 1, 2
STACK_BIOR15, STACK_DCT = 0, 1
BM_AUTO, BM_SHIFT, BM_CORR = 0, 1, 2
PROBE_FP64, PROBE_MFMA_I8, PROBE_MFMA_BF16 = 0, 1, 2
HT_STACK, HT_RECOMPUTE = 0, 1


class Params(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("patch", ctypes.c_int32),
        ("step", ctypes.c_int32),
        ("search", ctypes.c_int32),
        ("k_ht", ctypes.c_int32),
        ("k_wiener", ctypes.c_int32),
        ("ht_a", ctypes.c_float),
        ("ht_b", ctypes.c_float),
        ("ht_weight", ctypes.c_int32),
        ("tv_eps_rel", ctypes.c_float),
        ("keep_dc", ctypes.c_int32),
        ("bm_split", ctypes.c_int32),
        ("bm_method", ctypes.c_int32),
        ("ht_source", ctypes.c_int32),
    ]


class Image(ctypes.Structure):
    _fields_ = [
        ("noisy", ctypes.c_void_p),
        ("pilot", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("H", ctypes.c_int32),
        ("W", ctypes.c_int32),
        ("sigma", ctypes.c_float),
    ]


class GlobalParams(ctypes.Structure):
    _fields_ = [
        ("struct_size", ctypes.c_uint32),
        ("patch", ctypes.c_int32),
        ("search", ctypes.c_int32),
        ("k", ctypes.c_int32),
        ("levels", ctypes.c_int32),
        ("cycles", ctypes.c_int32),
        ("n_shifts", ctypes.c_int32),
        ("shifts", ctypes.c_int32 * 4),
        ("ht_a", ctypes.c_float),
        ("ht_b", ctypes.c_float),
        ("tv_eps_rel", ctypes.c_float),
    ]


class GBM3DError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"gbm3d status {status}: {msg}")
        self.status = status


_lib = None

_P = ctypes.c_void_p
_I = ctypes.c_int
_F = ctypes.c_float

_SIGNATURES = {
    "gbm3d_default_params": (None, [ctypes.POINTER(Params)]),
    "gbm3d_create": (_I, [ctypes.POINTER(_P), _I]),
    "gbm3d_destroy": (None, [_P]),
    "gbm3d_status_str": (ctypes.c_char_p, [_I]),
    "gbm3d_last_error": (ctypes.c_char_p, [_P]),
    "gbm3d_n_refs": (ctypes.c_int64, [_I, _I, _I]),
    "gbm3d_check_args": (_I, [_I, _I, _F, ctypes.POINTER(Params)]),
    "gbm3d_version": (ctypes.c_char_p, []),
    "gbm3d_match": (_I, [_P, _P, _I, _I, _I, ctypes.POINTER(Params), _P, _P]),
    "gbm3d_stack": (_I, [_P, _P, _I, _I, _I, _P, _P]),
    "gbm3d_basic": (_I, [_P, _P, _I, _I, _F, ctypes.POINTER(Params), _P, _P]),
    "gbm3d_wiener": (_I, [_P, _P, _P, _I, _I, _F, ctypes.POINTER(Params), _P, _P]),
    "gbm3d_denoise": (_I, [_P, _P, _I, _I, _F, ctypes.POINTER(Params), _P, _P, _P, _P]),
    "gbm3d_denoise_noalloc": (_I, [_P, _P, _I, _I, _F, ctypes.POINTER(Params), _P, _P, _P, _P]),
    "gbm3d_quantize": (_I, [_P, _P, _P, ctypes.c_size_t, _P]),
    "gbm3d_denoise_batch": (_I, [_P, ctypes.POINTER(Image), _I, ctypes.POINTER(Params), _I, _P]),
    "gbm3d_pilot_param_count": (_I, []),
    "gbm3d_pilot_load": (_I, [_P, _P, _P]),
    "gbm3d_pilot_infer": (_I, [_P, _P, _I, _I, _I, _P, _P, _P, _P]),
    "gbm3d_pilot_grad": (_I, [_P, _P, _P, _I, _I, _I, _P, _P, _P, _P, _P]),
    "gbm3d_pilot_adam": (_I, [_P, _P, _P, _P, _P, _I, _F, _F, _F, _F, _P]),
    "gbm3d_timing_enable": (_I, [_P, _I]),
    "gbm3d_timing_read": (_I, [_P, ctypes.c_char_p, ctypes.POINTER(ctypes.c_double),
                               ctypes.POINTER(ctypes.c_int64)]),
    "gbm3d_timing_reset": (_I, [_P]),
    "gbm3d_autotune": (_I, [_P, _P, _I, _I, _I, ctypes.POINTER(Params), _I, ctypes.POINTER(_I), ctypes.POINTER(_I),
                            ctypes.POINTER(_F), _P]),
    "gbm3d_tune_save": (_I, [_P, ctypes.c_char_p]),
    "gbm3d_tune_load": (_I, [_P, ctypes.c_char_p]),
    "gbm3d_global_default_params": (None, [ctypes.POINTER(GlobalParams)]),
    "gbm3d_global_basic": (_I, [_P, _P, _I, _I, _F, ctypes.POINTER(GlobalParams), _P, _P]),
    "gbm3d_global_match": (_I, [_P, _P, _I, _I, ctypes.POINTER(GlobalParams), _P, _P]),
    "gbm3d_probe": (_I, [_P, _I, _I, _I, _P, _P]),
    "gbm3d_probe_ops": (ctypes.c_double, [_I, _I, _I]),
}


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(python -m paper_2103_10765_amd.build)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in _SIGNATURES.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def default_params(**overrides) -> Params:
    p = Params()
    lib().gbm3d_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def global_default_params(**overrides) -> GlobalParams:
    """Global stage-1 parameters; `shifts` may be given as a sequence."""
    p = GlobalParams()
    lib().gbm3d_global_default_params(ctypes.byref(p))
    for k, v in overrides.items():
        if k == "shifts":
            v = list(v)
            p.n_shifts = len(v)
            for i in range(4):
                p.shifts[i] = int(v[i]) if i < len(v) else 0
            continue
        if not hasattr(p, k):
            raise KeyError(k)
        setattr(p, k, v)
    return p


def pilot_param_count() -> int:
    return int(lib().gbm3d_pilot_param_count())


def n_refs(H: int, W: int, step: int = 3) -> int:
    return int(lib().gbm3d_n_refs(H, W, step))


def check_args(H: int, W: int, sigma: float, params: Params | None = None) -> int:
    return int(lib().gbm3d_check_args(H, W, sigma, ctypes.byref(params) if params is not None else None))


def last_thread_error() -> str:
    return lib().gbm3d_last_error(None).decode()


def _stream(stream) -> ctypes.c_void_p:
    if stream is None:
        stream = torch.cuda.current_stream()
    return ctypes.c_void_p(stream.cuda_stream if hasattr(stream, "cuda_stream") else int(stream))


def _dev(t: torch.Tensor, dtype: torch.dtype, name: str) -> ctypes.c_void_p:
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    return ctypes.c_void_p(t.data_ptr())


def _hw(t: torch.Tensor):
    if t.dim() != 2:
        raise ValueError("images are 2-D [H, W]")
    return int(t.shape[0]), int(t.shape[1])


class Context:
    """One library context (device workspace) on a HIP device."""

    def __init__(self, device: int | None = None):
        if device is None:
            device = torch.cuda.current_device()
        self.device = int(device)
        h = ctypes.c_void_p()
        s = lib().gbm3d_create(ctypes.byref(h), self.device)
        if s != OK:
            raise GBM3DError(s, last_thread_error())
        self._h = h

    def close(self):
        if getattr(self, "_h", None) is not None and self._h.value:
            lib().gbm3d_destroy(self._h)
            self._h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def _check(self, s: int):
        if s != OK:
            raise GBM3DError(s, lib().gbm3d_last_error(self._h).decode())

    def _params(self, params):
        return ctypes.byref(params if params is not None else default_params())

    # -- entry points ------------------------------------------------------
    def match(self, img: torch.Tensor, K: int, params: Params | None = None, out=None, stream=None,
              split: int | None = None, method: int | None = None):
        H, W = _hw(img)
        p = params if params is not None else default_params()
        if split is not None or method is not None:
            p = Params.from_buffer_copy(p)
            if split is not None:
                p.bm_split = split
            if method is not None:
                p.bm_method = method
        n = n_refs(H, W, p.step)
        if out is None:
            out = torch.empty((n, K), dtype=torch.int16, device=img.device)
        self._check(lib().gbm3d_match(self._h, _dev(img, torch.uint16, "img"), H, W, K, ctypes.byref(p),
                                      _dev(out, torch.int16, "idx"), _stream(stream)))
        return out

    def stack(self, img: torch.Tensor, kind: int = STACK_BIOR15, out=None, stream=None):
        H, W = _hw(img)
        if out is None:
            out = torch.empty((H * W, 64), dtype=torch.float32, device=img.device)
        self._check(lib().gbm3d_stack(self._h, _dev(img, torch.uint16, "img"), H, W, kind,
                                      _dev(out, torch.float32, "out"), _stream(stream)))
        return out

    def basic(self, noisy: torch.Tensor, sigma: float, params: Params | None = None, out=None, stream=None):
        H, W = _hw(noisy)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
        self._check(lib().gbm3d_basic(self._h, _dev(noisy, torch.uint16, "noisy"), H, W, float(sigma),
                                      self._params(params), _dev(out, torch.float32, "out"), _stream(stream)))
        return out

    def wiener(self, noisy: torch.Tensor, pilot: torch.Tensor, sigma: float, params: Params | None = None,
               out=None, stream=None):
        H, W = _hw(noisy)
        if tuple(pilot.shape) != (H, W):
            raise ValueError("pilot shape differs from noisy")
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
        self._check(lib().gbm3d_wiener(self._h, _dev(noisy, torch.uint16, "noisy"),
                                       _dev(pilot, torch.uint16, "pilot"), H, W, float(sigma),
                                       self._params(params), _dev(out, torch.float32, "out"), _stream(stream)))
        return out

    def denoise(self, noisy: torch.Tensor, sigma: float, params: Params | None = None, out=None,
                basic_out=None, q_out=None, stream=None):
        H, W = _hw(noisy)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
        b = _dev(basic_out, torch.float32, "basic_out") if basic_out is not None else None
        q = _dev(q_out, torch.uint16, "q_out") if q_out is not None else None
        self._check(lib().gbm3d_denoise(self._h, _dev(noisy, torch.uint16, "noisy"), H, W, float(sigma),
                                        self._params(params), _dev(out, torch.float32, "out"), b, q,
                                        _stream(stream)))
        return out

    def denoise_noalloc(self, noisy: torch.Tensor, sigma: float, params: Params | None = None, out=None,
                        basic_out=None, q_out=None, stream=None):
        """denoise() with every intermediate buffer in the library's static
        device scratch (no device allocation inside the call).  `out` must be
        given when the caller cannot allocate either."""
        H, W = _hw(noisy)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
        b = _dev(basic_out, torch.float32, "basic_out") if basic_out is not None else None
        q = _dev(q_out, torch.uint16, "q_out") if q_out is not None else None
        self._check(lib().gbm3d_denoise_noalloc(self._h, _dev(noisy, torch.uint16, "noisy"), H, W, float(sigma),
                                                self._params(params), _dev(out, torch.float32, "out"), b, q,
                                                _stream(stream)))
        return out

    def denoise_batch(self, noisy, sigmas, pilots=None, outs=None, params: Params | None = None,
                      graph: bool = False, basic_only: bool = False, stream=None):
        """Denoise a list of uint16 CUDA images of any sizes in one batch.

        pilots: optional list (entries may be None) of uint16 pilots for stage 2;
        basic_only: stage 1 only.  Returns the list of float32 outputs."""
        n = len(noisy)
        if len(sigmas) != n:
            raise ValueError("one sigma per image")
        pilots = pilots if pilots is not None else [None] * n
        if outs is None:
            outs = [torch.empty(x.shape, dtype=torch.float32, device=x.device) for x in noisy]
        arr = (Image * max(n, 1))()
        for i, (x, s, pl, o) in enumerate(zip(noisy, sigmas, pilots, outs)):
            H, W = _hw(x)
            arr[i].noisy = _dev(x, torch.uint16, "noisy").value
            arr[i].pilot = _dev(pl, torch.uint16, "pilot").value if pl is not None else None
            if pl is not None and tuple(pl.shape) != (H, W):
                raise ValueError("pilot shape differs from noisy")
            if tuple(o.shape) != (H, W):
                raise ValueError("output shape differs from noisy")
            arr[i].out = _dev(o, torch.float32, "out").value
            arr[i].H, arr[i].W, arr[i].sigma = H, W, float(s)
        flags = (BATCH_GRAPH if graph else 0) | (BATCH_BASIC_ONLY if basic_only else 0)
        self._check(lib().gbm3d_denoise_batch(self._h, arr, n, self._params(params), flags, _stream(stream)))
        return outs

    def global_basic(self, noisy: torch.Tensor, sigma: float, params: GlobalParams | None = None, out=None,
                     stream=None):
        """Global stage 1 (volume form) of a uint16 CUDA image."""
        H, W = _hw(noisy)
        if out is None:
            out = torch.empty((H, W), dtype=torch.float32, device=noisy.device)
        p = params if params is not None else global_default_params()
        self._check(lib().gbm3d_global_basic(self._h, _dev(noisy, torch.uint16, "noisy"), H, W, float(sigma),
                                             ctypes.byref(p), _dev(out, torch.float32, "out"), _stream(stream)))
        return out

    def global_match(self, img: torch.Tensor, params: GlobalParams | None = None, stream=None):
        """Tile matching of the global stage 1: int16 [(H/patch)(W/patch), k]."""
        H, W = _hw(img)
        p = params if params is not None else global_default_params()
        out = torch.empty(((H // p.patch) * (W // p.patch), p.k), dtype=torch.int16, device=img.device)
        self._check(lib().gbm3d_global_match(self._h, _dev(img, torch.uint16, "img"), H, W, ctypes.byref(p),
                                             _dev(out, torch.int16, "idx"), _stream(stream)))
        return out

    # -- learned pilot -----------------------------------------------------
    def pilot_load(self, master: torch.Tensor, stream=None):
        if master.numel() != pilot_param_count():
            raise ValueError("master vector has the wrong length")
        self._check(lib().gbm3d_pilot_load(self._h, _dev(master, torch.float32, "master"), _stream(stream)))

    def pilot_infer(self, noisy: torch.Tensor, sigma: torch.Tensor, u16: bool = True, f32: bool = False,
                    stream=None):
        """noisy: [B, H, W] uint16 CUDA; sigma: [B] float32 CUDA.  Returns (u16, f32) outputs."""
        if noisy.dim() != 3:
            raise ValueError("noisy must be [B, H, W]")
        B, H, W = (int(v) for v in noisy.shape)
        if sigma.numel() != B:
            raise ValueError("one sigma per image")
        pu = torch.empty((B, H, W), dtype=torch.uint16, device=noisy.device) if u16 else None
        pf = torch.empty((B, H, W), dtype=torch.float32, device=noisy.device) if f32 else None
        self._check(lib().gbm3d_pilot_infer(self._h, _dev(noisy, torch.uint16, "noisy"), B, H, W,
                                            _dev(sigma, torch.float32, "sigma"),
                                            _dev(pu, torch.uint16, "pilot_u16") if pu is not None else None,
                                            _dev(pf, torch.float32, "pilot_f32") if pf is not None else None,
                                            _stream(stream)))
        return pu, pf

    def pilot_grad(self, noisy: torch.Tensor, target: torch.Tensor, sigma: torch.Tensor, grad=None, loss=None,
                   stream=None, weight: torch.Tensor | None = None):
        B, H, W = (int(v) for v in noisy.shape)
        if tuple(target.shape) != (B, H, W) or sigma.numel() != B:
            raise ValueError("shape mismatch")
        if weight is not None and weight.numel() != B:
            raise ValueError("weight needs one value per image")
        if grad is None:
            grad = torch.empty(pilot_param_count(), dtype=torch.float32, device=noisy.device)
        if loss is None:
            loss = torch.empty(1, dtype=torch.float32, device=noisy.device)
        self._check(lib().gbm3d_pilot_grad(self._h, _dev(noisy, torch.uint16, "noisy"),
                                           _dev(target, torch.float32, "target"), B, H, W,
                                           _dev(sigma, torch.float32, "sigma"),
                                           None if weight is None else _dev(weight, torch.float32, "weight"),
                                           _dev(grad, torch.float32, "grad"),
                                           _dev(loss, torch.float32, "loss"), _stream(stream)))
        return grad, loss

    def pilot_adam(self, master, m, v, grad, step: int, lr: float, beta1=0.9, beta2=0.999, eps=1e-8, stream=None):
        self._check(lib().gbm3d_pilot_adam(self._h, _dev(master, torch.float32, "master"),
                                           _dev(m, torch.float32, "m"), _dev(v, torch.float32, "v"),
                                           _dev(grad, torch.float32, "grad"), int(step), float(lr), float(beta1),
                                           float(beta2), float(eps), _stream(stream)))

    def timing(self, on: bool = True):
        self._check(lib().gbm3d_timing_enable(self._h, 1 if on else 0))

    def timing_reset(self):
        self._check(lib().gbm3d_timing_reset(self._h))

    def timing_read(self, kernel: str):
        """(total milliseconds, launches) of one kernel since the last reset."""
        ms = ctypes.c_double()
        n = ctypes.c_int64()
        self._check(lib().gbm3d_timing_read(self._h, kernel.encode(), ctypes.byref(ms), ctypes.byref(n)))
        return ms.value, n.value

    def autotune(self, img: torch.Tensor, K: int, reps: int = 3, params: Params | None = None, stream=None):
        """Times every block-matching variant on img (and, for K == k_ht <= 16,
        both stage-1 group-kernel shapes) and records the fastest for its
        (K, search, shape class); returns (method, split, ms per matching run)."""
        H, W = _hw(img)
        m, sp, ms = _I(), _I(), _F()
        self._check(lib().gbm3d_autotune(self._h, _dev(img, torch.uint16, "img"), H, W, K,
                                         ctypes.byref(params) if params is not None else None, reps,
                                         ctypes.byref(m), ctypes.byref(sp), ctypes.byref(ms), _stream(stream)))
        return m.value, sp.value, ms.value

    def tune_save(self, path: str):
        self._check(lib().gbm3d_tune_save(self._h, os.fsencode(path)))

    def tune_load(self, path: str):
        self._check(lib().gbm3d_tune_load(self._h, os.fsencode(path)))

    def quantize(self, x: torch.Tensor, out=None, stream=None):
        if out is None:
            out = torch.empty(x.shape, dtype=torch.uint16, device=x.device)
        self._check(lib().gbm3d_quantize(self._h, _dev(x, torch.float32, "in"), _dev(out, torch.uint16, "out"),
                                         x.numel(), _stream(stream)))
        return out

    def probe(self, kind: int, blocks: int, iters: int, sink=None, stream=None):
        """One peak-rate probe launch (PROBE_FP64 / PROBE_MFMA_I8 /
        PROBE_MFMA_BF16); returns (sink, arithmetic operations of the launch)."""
        if sink is None:
            sink = torch.empty(blocks * 256, dtype=torch.float32, device=torch.device("cuda", self.device))
        if sink.numel() < blocks * 256:
            raise ValueError("sink needs blocks * 256 floats")
        self._check(lib().gbm3d_probe(self._h, kind, blocks, iters, _dev(sink, torch.float32, "sink"),
                                      _stream(stream)))
        return sink, float(lib().gbm3d_probe_ops(kind, blocks, iters))


_default_ctx: dict[int, Context] = {}


def context(device: int | None = None) -> Context:
    if device is None:
        device = torch.cuda.current_device()
    if device not in _default_ctx:
        _default_ctx[device] = Context(device)
    return _default_ctx[device]


def denoise(noisy: torch.Tensor, sigma: float, params: Params | None = None) -> torch.Tensor:
    """Two-stage G-BM3D of a uint16 CUDA image; returns float32 [H, W]."""
    return context(noisy.device.index).denoise(noisy, sigma, params)


def basic(noisy: torch.Tensor, sigma: float, params: Params | None = None) -> torch.Tensor:
    """Stage 1 only (basic estimate)."""
    return context(noisy.device.index).basic(noisy, sigma, params)


def psnr_db(Y, clean) -> float:
    """10 log10(1 / MSE) of clip(Y, 0, 1) against a clean [0, 1] image (NumPy arrays)."""
    import numpy as np
    Y = np.clip(np.asarray(Y, dtype=np.float64), 0.0, 1.0)
    mse = float(np.mean((Y - np.asarray(clean, dtype=np.float64)) ** 2))
    return 10.0 * np.log10(1.0 / mse)
