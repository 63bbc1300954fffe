"""Python binding of the C ABI in include/nrc.h (argument marshalling only).

Every function named ``nrc_*`` here calls the C entry point of the same name
with device pointers taken from torch tensors and the current HIP stream; all
arithmetic happens in the HIP kernels of libnrc.so.  PyTorch only provides
device memory and streams.  Importing this module fails loudly when the
library has not been built (``python -m paper_2106_12372_amd.build``).
"""
from __future__ import annotations

import ctypes
import os
import sys
from ctypes import POINTER, c_double, c_float, c_int, c_int32, c_int64, c_size_t, c_uint64, c_void_p
from typing import Optional

import numpy as np

_LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libnrc.so")
if not os.path.exists(_LIB_PATH):
    raise ImportError(f"{_LIB_PATH} is missing: build it with `python -m paper_2106_12372_amd.build`")
lib = ctypes.CDLL(_LIB_PATH)

# Status codes, precisions, presets and layouts (same values as nrc.h).
NRC_OK, NRC_PENDING, NRC_EINVAL, NRC_ENOMEM, NRC_EDEVICE, NRC_EBUSY, NRC_ENOTFOUND = 0, 1, -1, -2, -3, -4, -5
NRC_FP32, NRC_FP16, NRC_BF16, NRC_FP32_VALU = 0, 1, 2, 3
NRC_PRESET_CONFIG, NRC_PRESET_PAPER, NRC_PRESET_PAPER_TRI, NRC_PRESET_PAPER_GAUSS = 0, 1, 2, 3
NRC_RAW14, NRC_RAW16 = 0, 1
NRC_REQ_INFER, NRC_REQ_TRAIN = 0, 1
ENC_WIDTH = 64
NRC_NOALLOC_SCRATCH_BYTES = 48 << 20   # the fixed scratch array of nrc_train_step_noalloc
PRECISIONS = {"fp32": NRC_FP32, "fp16": NRC_FP16, "bf16": NRC_BF16, "fp32_valu": NRC_FP32_VALU}


class NrcError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"nrc error {code}: {msg}")
        self.code = code


class nrc_config(ctypes.Structure):
    _fields_ = [("width", c_int32), ("n_hidden", c_int32), ("n_out", c_int32),
                ("precision", c_int32), ("enc_preset", c_int32), ("lr", c_float),
                ("beta1", c_float), ("beta2", c_float), ("adam_eps", c_float),
                ("loss_eps", c_float), ("loss_scale", c_float), ("ema_alpha", c_float),
                ("factorize", c_int32),
                ("seed", c_uint64)]


class nrc_serve_config(ctypes.Structure):
    _fields_ = [("n_caches", c_int32), ("cache_cfg", nrc_config), ("arena", c_void_p),
                ("arena_bytes", c_size_t), ("n_streams", c_int32), ("max_inflight", c_int32)]


class nrc_request(ctypes.Structure):
    _fields_ = [("kind", c_int32), ("enc", c_void_p), ("target", c_void_p), ("rgb", c_void_p),
                ("n", c_int64)]


class nrc_result(ctypes.Structure):
    _fields_ = [("status", c_int32), ("skipped", c_int32), ("loss", c_float),
                ("t_submit", c_double), ("t_start", c_double), ("t_done", c_double)]


def _decl(name, restype, *argtypes):
    if not hasattr(lib, name):
        return None
    fn = getattr(lib, name)
    fn.restype = restype
    fn.argtypes = list(argtypes)
    return fn


_P = c_void_p
_decl("nrc_config_default", c_int, POINTER(nrc_config))
_decl("nrc_last_error", ctypes.c_char_p)
_decl("nrc_param_count", c_int64, POINTER(nrc_config))
_decl("nrc_cache_bytes", c_size_t, POINTER(nrc_config))
_decl("nrc_train_scratch_bytes", c_size_t, POINTER(nrc_config), c_int64)
_decl("nrc_enc_elem_bytes", c_int, POINTER(nrc_config))
_decl("nrc_cache_create", c_int, POINTER(nrc_config), _P, c_size_t, _P, POINTER(_P))
_decl("nrc_cache_destroy", c_int, _P)
_decl("nrc_cache_config", c_int, _P, POINTER(nrc_config))
_decl("nrc_set_weights", c_int, _P, POINTER(c_float), c_int64, _P)
_decl("nrc_get_weights", c_int, _P, POINTER(c_float), c_int64, _P)
_decl("nrc_set_weights_device", c_int, _P, _P, c_int64, _P)
_decl("nrc_get_state", c_int, _P, POINTER(c_float), POINTER(c_float), POINTER(c_float), c_int64,
      POINTER(c_int64), _P)
_decl("nrc_set_state", c_int, _P, POINTER(c_float), POINTER(c_float), POINTER(c_float), c_int64,
      c_int64, _P)
_decl("nrc_get_ema", c_int, _P, POINTER(c_float), POINTER(c_float), c_int64, _P)
_decl("nrc_set_ema", c_int, _P, POINTER(c_float), POINTER(c_float), c_int64, _P)
_decl("nrc_encode", c_int, _P, _P, c_int, c_int64, _P, _P)
_decl("nrc_forward", c_int, _P, _P, c_int64, _P, _P)
_decl("nrc_forward_raw", c_int, _P, _P, c_int, c_int64, _P, _P)
_decl("nrc_train_step", c_int, _P, _P, _P, c_int64, _P, c_size_t, _P, _P, _P)
_decl("nrc_train_step_noalloc", c_int, _P, _P, _P, c_int64, _P, _P, _P)
_decl("nrc_act_ws_bytes", c_size_t, POINTER(nrc_config), c_int64)
_decl("nrc_forward_train", c_int, _P, _P, c_int64, _P, c_size_t, _P, _P)
_decl("nrc_backward", c_int, _P, _P, _P, _P, c_int64, _P, c_size_t, _P, _P, _P)
_decl("nrc_shuffle_scratch_bytes", c_size_t, c_int64)
_decl("nrc_shuffle", c_int, c_int64, c_uint64, _P, _P, c_size_t, _P)
_decl("nrc_train_step_indexed", c_int, _P, _P, _P, _P, c_int64, _P, c_size_t, _P, _P, _P)
_decl("nrc_frame_scratch_bytes", c_size_t, POINTER(nrc_config), c_int64, c_int, c_int64)
_decl("nrc_train_frame", c_int, _P, _P, _P, c_int64, c_int, c_int64, c_uint64, _P, c_size_t, _P, _P, _P)
_decl("nrc_train_frame_indexed", c_int, _P, _P, _P, _P, c_int64, c_int, c_int64, _P, c_size_t, _P, _P, _P)
_decl("nrc_train_frame_raw", c_int, _P, _P, c_int, _P, c_int64, c_int, c_int64, c_uint64, _P, c_size_t, _P, _P, _P)
_decl("nrc_self_training_targets", c_int, _P, _P, _P, _P, c_int64, c_int64, _P, _P)
_decl("nrc_error_norms_scratch_bytes", c_size_t, c_int64)
_decl("nrc_error_norms", c_int, _P, _P, c_int64, _P, c_size_t, _P, _P)
_decl("nrc_serve_create", c_int, POINTER(nrc_serve_config), POINTER(_P))
_decl("nrc_serve_set_weights", c_int, _P, c_int, POINTER(c_float), c_int64)
_decl("nrc_serve_get_weights", c_int, _P, c_int, POINTER(c_float), c_int64)
_decl("nrc_serve_submit", c_int, _P, c_int, POINTER(nrc_request), POINTER(c_uint64))
_decl("nrc_serve_poll", c_int, _P, c_uint64, POINTER(nrc_result))
_decl("nrc_serve_drain", c_int, _P)
_decl("nrc_serve_destroy", c_int, _P)

EXPORTED = ["nrc_config_default", "nrc_last_error", "nrc_param_count", "nrc_cache_bytes",
            "nrc_train_scratch_bytes", "nrc_enc_elem_bytes", "nrc_cache_create", "nrc_cache_destroy",
            "nrc_cache_config", "nrc_set_weights", "nrc_get_weights", "nrc_set_weights_device",
            "nrc_get_state", "nrc_set_state", "nrc_get_ema", "nrc_set_ema", "nrc_encode", "nrc_forward", "nrc_forward_raw", "nrc_train_step",
            "nrc_train_step_noalloc",
            "nrc_act_ws_bytes", "nrc_forward_train", "nrc_backward", "nrc_shuffle_scratch_bytes", "nrc_shuffle", "nrc_train_step_indexed",
            "nrc_frame_scratch_bytes", "nrc_train_frame", "nrc_train_frame_indexed", "nrc_train_frame_raw", "nrc_self_training_targets", "nrc_error_norms_scratch_bytes", "nrc_error_norms", "nrc_serve_create", "nrc_serve_set_weights", "nrc_serve_get_weights",
            "nrc_serve_submit", "nrc_serve_poll", "nrc_serve_drain", "nrc_serve_destroy"]


def last_error() -> str:
    return lib.nrc_last_error().decode()


def check(rc: int) -> int:
    if rc < 0:
        raise NrcError(rc, last_error())
    return rc


# ---------------------------------------------------------------------------
# Configuration
# ---------------------------------------------------------------------------
def make_config(width: int = 64, n_hidden: int = 5, precision="fp16", enc_preset: int = NRC_PRESET_CONFIG,
                lr: float = 1e-2, beta1: float = 0.9, beta2: float = 0.99, adam_eps: float = 1e-8,
                loss_eps: float = 0.01, loss_scale: Optional[float] = None,
                ema_alpha: float = 0.0, factorize: bool = False) -> nrc_config:
    cfg = nrc_config()
    check(lib.nrc_config_default(ctypes.byref(cfg)))
    prec = PRECISIONS[precision] if isinstance(precision, str) else int(precision)
    cfg.width, cfg.n_hidden, cfg.precision, cfg.enc_preset = width, n_hidden, prec, enc_preset
    cfg.lr, cfg.beta1, cfg.beta2, cfg.adam_eps, cfg.loss_eps = lr, beta1, beta2, adam_eps, loss_eps
    cfg.loss_scale = (1.0 if prec in (NRC_FP32, NRC_FP32_VALU) else 128.0) if loss_scale is None else loss_scale
    cfg.ema_alpha = ema_alpha
    cfg.factorize = 1 if factorize else 0
    return cfg


def _torch():
    import torch
    return torch


def enc_dtype(cfg: nrc_config):
    torch = _torch()
    return {NRC_FP32: torch.float32, NRC_FP16: torch.float16, NRC_BF16: torch.bfloat16,
            NRC_FP32_VALU: torch.float32}[cfg.precision]


def _stream(stream) -> c_void_p:
    if stream is None:
        return c_void_p(_torch().cuda.current_stream().cuda_stream)
    if isinstance(stream, int):
        return c_void_p(stream)
    return c_void_p(stream.cuda_stream)


def _keep(stream, *tensors):
    """Tensors this binding allocated on the current stream but hands to work on
    `stream`: tell torch's caching allocator that they are in use there, so it
    does not reuse their memory before that stream's work has finished."""
    if stream is None:
        return
    torch = _torch()
    s = torch.cuda.ExternalStream(stream) if isinstance(stream, int) else stream
    if s == torch.cuda.current_stream(s.device):
        return
    for t in tensors:
        if t is not None:
            t.record_stream(s)


def _ptr(t) -> c_void_p:
    return c_void_p(0 if t is None else t.data_ptr())


def _need(t, dtype, shape_tail, name):
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if t.dtype != dtype:
        raise ValueError(f"{name} must be {dtype}, got {t.dtype}")
    if tuple(t.shape[1:]) != tuple(shape_tail):
        raise ValueError(f"{name} must have shape [n]{list(shape_tail)}, got {list(t.shape)}")


# ---------------------------------------------------------------------------
# Entry points (same names as the C ABI)
# ---------------------------------------------------------------------------
def nrc_param_count(cfg: nrc_config) -> int:
    return check(lib.nrc_param_count(ctypes.byref(cfg)))


def nrc_cache_bytes(cfg: nrc_config) -> int:
    b = lib.nrc_cache_bytes(ctypes.byref(cfg))
    if b == 0:
        raise NrcError(NRC_EINVAL, last_error())
    return b


def nrc_train_scratch_bytes(cfg: nrc_config, n: int) -> int:
    b = lib.nrc_train_scratch_bytes(ctypes.byref(cfg), n)
    if b == 0:
        raise NrcError(NRC_EINVAL, last_error())
    return b


class Cache:
    """One radiance cache: a handle plus its device workspace (a torch tensor)."""

    def __init__(self, cfg: nrc_config, device=None, stream=None):
        torch = _torch()
        self.cfg = cfg
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        nbytes = nrc_cache_bytes(cfg)
        # 256 bytes of slack so the workspace can be aligned to 256
        self._ws_t = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._ws_t.data_ptr()) % 256
        self.ws = self._ws_t[off:off + nbytes]
        handle = c_void_p()
        check(lib.nrc_cache_create(ctypes.byref(cfg), c_void_p(self.ws.data_ptr()), nbytes,
                                   _stream(stream), ctypes.byref(handle)))
        self.handle = handle
        self.n_params = nrc_param_count(cfg)
        self._scratch = None

    def __del__(self, _finalizing=sys.is_finalizing):
        # at interpreter exit the module's globals may already be gone (the
        # default argument keeps the check itself alive); the process ends and
        # the driver reclaims the device memory
        if _finalizing() or lib is None:
            return
        h = getattr(self, "handle", None)
        if h is not None and h.value:
            lib.nrc_cache_destroy(h)
            self.handle = None

    @property
    def enc_dtype(self):
        return enc_dtype(self.cfg)

    def scratch(self, n: int):
        torch = _torch()
        need = nrc_train_scratch_bytes(self.cfg, n)
        if self._scratch is None or self._scratch[1] < need:
            t = torch.empty(need + 256, dtype=torch.uint8, device=self.device)
            off = (-t.data_ptr()) % 256
            self._scratch = (t, need, off)
        t, size, off = self._scratch
        return t[off:off + size], size

    # weights and state ------------------------------------------------------
    def set_weights(self, w, stream=None):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        check(lib.nrc_set_weights(self.handle, w.ctypes.data_as(POINTER(c_float)), w.size, _stream(stream)))

    def set_weights_device(self, w, stream=None):
        _need(w.reshape(-1, 1), _torch().float32, (1,), "weights")
        check(lib.nrc_set_weights_device(self.handle, _ptr(w), w.numel(), _stream(stream)))

    def get_weights(self, stream=None) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(lib.nrc_get_weights(self.handle, out.ctypes.data_as(POINTER(c_float)), out.size, _stream(stream)))
        return out

    def get_state(self, stream=None):
        w, m, v = (np.empty(self.n_params, dtype=np.float32) for _ in range(3))
        t = c_int64()
        fp = lambda a: a.ctypes.data_as(POINTER(c_float))
        check(lib.nrc_get_state(self.handle, fp(w), fp(m), fp(v), self.n_params, ctypes.byref(t), _stream(stream)))
        return w, m, v, t.value

    def get_ema(self, stream=None):
        """(W_bar, E) of a cache created with ema_alpha > 0."""
        wb, e = (np.empty(self.n_params, dtype=np.float32) for _ in range(2))
        fp = lambda a: a.ctypes.data_as(POINTER(c_float))
        check(lib.nrc_get_ema(self.handle, fp(wb), fp(e), self.n_params, _stream(stream)))
        return wb, e

    def set_ema(self, w_bar, e, stream=None):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1)) for a in (w_bar, e)]
        fp = lambda a: a.ctypes.data_as(POINTER(c_float))
        check(lib.nrc_set_ema(self.handle, fp(arrs[0]), fp(arrs[1]), self.n_params, _stream(stream)))

    def set_state(self, w, m, v, t, stream=None):
        arrs = [np.ascontiguousarray(np.asarray(a, dtype=np.float32).reshape(-1)) for a in (w, m, v)]
        fp = lambda a: a.ctypes.data_as(POINTER(c_float))
        check(lib.nrc_set_state(self.handle, fp(arrs[0]), fp(arrs[1]), fp(arrs[2]), self.n_params, int(t),
                                _stream(stream)))


def nrc_encode(cache: Cache, raw, layout: int = NRC_RAW14, enc=None, stream=None):
    torch = _torch()
    width = 14 if layout == NRC_RAW14 else 16
    _need(raw, torch.float32, (width,), "raw")
    n = raw.shape[0]
    if enc is None:
        enc = torch.empty((n, ENC_WIDTH), dtype=cache.enc_dtype, device=raw.device)
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _keep(stream, enc)
    check(lib.nrc_encode(cache.handle, _ptr(raw), layout, n, _ptr(enc), _stream(stream)))
    return enc


def nrc_forward(cache: Cache, enc, rgb=None, stream=None):
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    n = enc.shape[0]
    if rgb is None:
        rgb = torch.empty((n, 3), dtype=torch.float32, device=enc.device)
    _need(rgb, torch.float32, (3,), "rgb")
    _keep(stream, rgb)
    check(lib.nrc_forward(cache.handle, _ptr(enc), n, _ptr(rgb), _stream(stream)))
    return rgb


def nrc_forward_raw(cache: Cache, raw, layout: int = NRC_RAW14, rgb=None, stream=None):
    """Fused encode + inference on raw records."""
    torch = _torch()
    width = 14 if layout == NRC_RAW14 else 16
    _need(raw, torch.float32, (width,), "raw")
    n = raw.shape[0]
    if rgb is None:
        rgb = torch.empty((n, 3), dtype=torch.float32, device=raw.device)
    _need(rgb, torch.float32, (3,), "rgb")
    _keep(stream, rgb)
    check(lib.nrc_forward_raw(cache.handle, _ptr(raw), layout, n, _ptr(rgb), _stream(stream)))
    return rgb


def nrc_train_step(cache: Cache, enc, target, loss=None, skipped=None, scratch=None, stream=None):
    """One Adam step on (enc, target); returns the device scalars (loss, skipped)."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(target, torch.float32, (3,), "target")
    n = enc.shape[0]
    if target.shape[0] != n:
        raise ValueError("enc and target differ in length")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=enc.device)
    if skipped is None:
        skipped = torch.empty(1, dtype=torch.int32, device=enc.device)
    sc, size = cache.scratch(n) if scratch is None else (scratch, scratch.numel())
    _keep(stream, loss, skipped, sc)
    check(lib.nrc_train_step(cache.handle, _ptr(enc), _ptr(target), n, _ptr(sc), size, _ptr(loss),
                             _ptr(skipped), _stream(stream)))
    return loss, skipped


def nrc_train_step_noalloc(cache: Cache, enc, target, loss=None, skipped=None, stream=None):
    """nrc_train_step on the library's fixed scratch array (no scratch buffer);
    returns the device scalars (loss, skipped)."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(target, torch.float32, (3,), "target")
    n = enc.shape[0]
    if target.shape[0] != n:
        raise ValueError("enc and target differ in length")
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=enc.device)
    if skipped is None:
        skipped = torch.empty(1, dtype=torch.int32, device=enc.device)
    _keep(stream, loss, skipped)
    check(lib.nrc_train_step_noalloc(cache.handle, _ptr(enc), _ptr(target), n, _ptr(loss), _ptr(skipped),
                                     _stream(stream)))
    return loss, skipped


def _aligned_bytes(nbytes: int, device):
    """A 256-byte aligned uint8 device buffer of nbytes."""
    torch = _torch()
    t = torch.empty(nbytes + 256, dtype=torch.uint8, device=device)
    off = (-t.data_ptr()) % 256
    return t[off:off + nbytes]


def nrc_shuffle(n: int, seed: int, device="cuda", perm=None, scratch=None, stream=None):
    """Shuffled record order (Sec. 3.5): int32 device tensor perm[n]."""
    torch = _torch()
    if perm is None:
        perm = torch.empty(n, dtype=torch.int32, device=device)
    sc = _aligned_bytes(max(1, lib.nrc_shuffle_scratch_bytes(n)), perm.device) if scratch is None else scratch
    _keep(stream, perm, sc)
    check(lib.nrc_shuffle(n, seed & (2 ** 64 - 1), _ptr(perm), _ptr(sc), sc.numel(), _stream(stream)))
    return perm


def nrc_train_step_indexed(cache: Cache, enc, target, idx, loss=None, skipped=None, stream=None):
    """One Adam step on records idx of (enc, target); returns the device scalars (loss, skipped)."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(target, torch.float32, (3,), "target")
    _need(idx, torch.int32, (), "idx")
    if target.shape[0] != enc.shape[0]:
        raise ValueError("enc and target differ in length")
    n = idx.shape[0]
    if loss is None:
        loss = torch.empty(1, dtype=torch.float32, device=enc.device)
    if skipped is None:
        skipped = torch.empty(1, dtype=torch.int32, device=enc.device)
    sc, size = cache.scratch(n)
    _keep(stream, loss, skipped, sc)
    check(lib.nrc_train_step_indexed(cache.handle, _ptr(enc), _ptr(target), _ptr(idx), n, _ptr(sc), size,
                                     _ptr(loss), _ptr(skipped), _stream(stream)))
    return loss, skipped


def nrc_frame_scratch_bytes(cfg: nrc_config, n_records: int, steps: int, batch: int) -> int:
    b = lib.nrc_frame_scratch_bytes(ctypes.byref(cfg), n_records, steps, batch)
    if b == 0:
        raise NrcError(NRC_EINVAL, last_error())
    return b


def nrc_train_frame(cache: Cache, enc, target, steps: int = 4, batch: int = 16384, seed: int = 0,
                    scratch=None, stream=None):
    """Shuffle the frame's records and run `steps` training steps on disjoint
    batches (Sec. 3.3 and 3.5); returns device tensors (losses[steps], skipped[steps])."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(target, torch.float32, (3,), "target")
    n = enc.shape[0]
    if target.shape[0] != n:
        raise ValueError("enc and target differ in length")
    if scratch is None:
        scratch = _aligned_bytes(nrc_frame_scratch_bytes(cache.cfg, n, steps, batch), enc.device)
    losses = torch.empty(steps, dtype=torch.float32, device=enc.device)
    skipped = torch.empty(steps, dtype=torch.int32, device=enc.device)
    _keep(stream, scratch, losses, skipped)
    check(lib.nrc_train_frame(cache.handle, _ptr(enc), _ptr(target), n, steps, batch, seed & (2 ** 64 - 1),
                              _ptr(scratch), scratch.numel(), _ptr(losses), _ptr(skipped), _stream(stream)))
    return losses, skipped


def nrc_train_frame_indexed(cache: Cache, enc, target, perm, steps: int = 4, batch: int = 16384,
                            scratch=None, stream=None):
    """The training steps of nrc_train_frame on a given permutation perm[n]
    (e.g. from nrc_shuffle on another stream); returns (losses[steps], skipped[steps])."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(target, torch.float32, (3,), "target")
    _need(perm, torch.int32, (), "perm")
    n = enc.shape[0]
    if target.shape[0] != n or perm.shape[0] != n:
        raise ValueError("enc, target and perm differ in length")
    if scratch is None:
        scratch = _aligned_bytes(nrc_frame_scratch_bytes(cache.cfg, n, steps, batch), enc.device)
    losses = torch.empty(steps, dtype=torch.float32, device=enc.device)
    skipped = torch.empty(steps, dtype=torch.int32, device=enc.device)
    _keep(stream, scratch, losses, skipped)
    check(lib.nrc_train_frame_indexed(cache.handle, _ptr(enc), _ptr(target), _ptr(perm), n, steps, batch,
                                      _ptr(scratch), scratch.numel(), _ptr(losses), _ptr(skipped),
                                      _stream(stream)))
    return losses, skipped


def nrc_train_frame_raw(cache: Cache, raw, target, layout: int = NRC_RAW14, steps: int = 4, batch: int = 16384,
                        seed: int = 0, scratch=None, stream=None):
    """nrc_train_frame on raw records (FP32 [n][14] or [n][16]), encoded inside
    the training kernels; returns (losses[steps], skipped[steps])."""
    torch = _torch()
    width = 14 if layout == NRC_RAW14 else 16
    _need(raw, torch.float32, (width,), "raw")
    _need(target, torch.float32, (3,), "target")
    n = raw.shape[0]
    if target.shape[0] != n:
        raise ValueError("raw and target differ in length")
    if scratch is None:
        scratch = _aligned_bytes(nrc_frame_scratch_bytes(cache.cfg, n, steps, batch), raw.device)
    losses = torch.empty(steps, dtype=torch.float32, device=raw.device)
    skipped = torch.empty(steps, dtype=torch.int32, device=raw.device)
    _keep(stream, scratch, losses, skipped)
    check(lib.nrc_train_frame_raw(cache.handle, _ptr(raw), layout, _ptr(target), n, steps, batch,
                                  seed & (2 ** 64 - 1), _ptr(scratch), scratch.numel(), _ptr(losses),
                                  _ptr(skipped), _stream(stream)))
    return losses, skipped


def nrc_self_training_targets(radiance, throughput, tail_rgb, tail_index, stream=None):
    """target = radiance + throughput * tail_rgb[tail_index] (Sec. 3.2 self-training)."""
    torch = _torch()
    _need(radiance, torch.float32, (3,), "radiance")
    _need(throughput, torch.float32, (3,), "throughput")
    _need(tail_rgb, torch.float32, (3,), "tail_rgb")
    _need(tail_index, torch.int32, (), "tail_index")
    n = radiance.shape[0]
    if throughput.shape[0] != n or tail_index.shape[0] != n:
        raise ValueError("radiance, throughput and tail_index differ in length")
    target = torch.empty((n, 3), dtype=torch.float32, device=radiance.device)
    _keep(stream, target)
    check(lib.nrc_self_training_targets(_ptr(radiance), _ptr(throughput), _ptr(tail_rgb), _ptr(tail_index), n,
                                        tail_rgb.shape[0], _ptr(target), _stream(stream)))
    return target


def nrc_act_ws_bytes(cfg: nrc_config, n: int) -> int:
    b = lib.nrc_act_ws_bytes(ctypes.byref(cfg), n)
    if b == 0 and n > 0:
        raise NrcError(NRC_EINVAL, last_error())
    return b


def nrc_forward_train(cache: Cache, enc, act=None, rgb=None, stream=None):
    """Predictions for enc with the training weights, keeping the activations
    for nrc_backward; returns (rgb[n][3], act) with act a uint8 device buffer."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    n = enc.shape[0]
    if rgb is None:
        rgb = torch.empty((n, 3), dtype=torch.float32, device=enc.device)
    if act is None:
        act = torch.empty(max(nrc_act_ws_bytes(cache.cfg, n), 16), dtype=torch.uint8, device=enc.device)
    _keep(stream, rgb, act)
    check(lib.nrc_forward_train(cache.handle, _ptr(enc), n, _ptr(act), act.numel(), _ptr(rgb), _stream(stream)))
    return rgb, act


def nrc_backward(cache: Cache, enc, grad_rgb, want_grad_enc: bool = True, act=None, scratch=None, stream=None):
    """Gradients of sum(grad_rgb * network(enc)) w.r.t. the weights and (optionally)
    enc; act: the buffer of nrc_forward_train for the same enc and weights, or
    None to recompute the forward pass."""
    torch = _torch()
    _need(enc, cache.enc_dtype, (ENC_WIDTH,), "enc")
    _need(grad_rgb, torch.float32, (3,), "grad_rgb")
    n = enc.shape[0]
    if act is not None and act.numel() < nrc_act_ws_bytes(cache.cfg, n):
        raise ValueError("activation buffer too small for this batch")
    grad_w = torch.empty(cache.n_params, dtype=torch.float32, device=enc.device)
    grad_enc = torch.empty((n, ENC_WIDTH), dtype=torch.float32, device=enc.device) if want_grad_enc else None
    sc, size = cache.scratch(n) if scratch is None else (scratch, scratch.numel())
    _keep(stream, grad_w, grad_enc, sc)
    check(lib.nrc_backward(cache.handle, _ptr(enc), _ptr(act), _ptr(grad_rgb), n, _ptr(sc), size, _ptr(grad_w),
                           _ptr(grad_enc), _stream(stream)))
    return grad_w, grad_enc


def nrc_error_norms(got, ref, stream=None):
    """Per-channel error norms of got [n][3] (FP32) against ref [n][3] (FP64),
    reduced in FP64 on the device: a [3][4] FP64 tensor of (sum (got-ref)^2,
    sum ref^2, max |got-ref|, max |ref|) per channel."""
    torch = _torch()
    _need(got, torch.float32, (3,), "got")
    _need(ref, torch.float64, (3,), "ref")
    n = got.shape[0]
    if ref.shape[0] != n:
        raise ValueError("got and ref differ in length")
    sc = torch.empty(lib.nrc_error_norms_scratch_bytes(n) // 8, dtype=torch.float64, device=got.device)
    out = torch.empty((3, 4), dtype=torch.float64, device=got.device)
    _keep(stream, sc, out)
    check(lib.nrc_error_norms(_ptr(got), _ptr(ref), n, _ptr(sc), sc.numel() * 8, _ptr(out), _stream(stream)))
    return out


# ---------------------------------------------------------------------------
# Serving
# ---------------------------------------------------------------------------
class Server:
    """Continuous-batching server over `n_caches` resident caches (nrc_serve_*).

    The arena (caches + per-request scratch) is one device tensor of
    `arena_bytes`.  Request tensors are kept alive here until their ticket has
    been collected by poll().  The server runs requests on its own streams and
    does not wait for work queued on others: a request's tensors must be
    complete (e.g. after torch.cuda.synchronize()) when it is submitted.
    """

    def __init__(self, n_caches: int, cfg: nrc_config, arena_bytes: int, n_streams: int = 4,
                 max_inflight: int = 64, device=None):
        torch = _torch()
        self.device = torch.device("cuda", torch.cuda.current_device()) if device is None else torch.device(device)
        self.cfg = cfg
        self._arena_t = torch.empty(arena_bytes + 256, dtype=torch.uint8, device=self.device)
        off = (-self._arena_t.data_ptr()) % 256
        sc = nrc_serve_config()
        sc.n_caches, sc.cache_cfg = n_caches, cfg
        sc.arena, sc.arena_bytes = self._arena_t.data_ptr() + off, arena_bytes
        sc.n_streams, sc.max_inflight = n_streams, max_inflight
        torch.cuda.synchronize(self.device)
        h = c_void_p()
        check(lib.nrc_serve_create(ctypes.byref(sc), ctypes.byref(h)))
        self.handle = h
        self.n_params = nrc_param_count(cfg)
        self._live = {}

    def set_weights(self, cache_id: int, w):
        w = np.ascontiguousarray(np.asarray(w, dtype=np.float32).reshape(-1))
        check(lib.nrc_serve_set_weights(self.handle, cache_id, w.ctypes.data_as(POINTER(c_float)), w.size))

    def get_weights(self, cache_id: int) -> np.ndarray:
        out = np.empty(self.n_params, dtype=np.float32)
        check(lib.nrc_serve_get_weights(self.handle, cache_id, out.ctypes.data_as(POINTER(c_float)), out.size))
        return out

    def _submit(self, cache_id, req, keep):
        t = c_uint64()
        check(lib.nrc_serve_submit(self.handle, cache_id, ctypes.byref(req), ctypes.byref(t)))
        self._live[t.value] = keep
        return t.value

    def submit_infer(self, cache_id: int, enc, rgb) -> int:
        torch = _torch()
        _need(enc, enc_dtype(self.cfg), (ENC_WIDTH,), "enc")
        _need(rgb, torch.float32, (3,), "rgb")
        req = nrc_request(NRC_REQ_INFER, enc.data_ptr(), None, rgb.data_ptr(), enc.shape[0])
        return self._submit(cache_id, req, (enc, rgb))

    def submit_train(self, cache_id: int, enc, target) -> int:
        torch = _torch()
        _need(enc, enc_dtype(self.cfg), (ENC_WIDTH,), "enc")
        _need(target, torch.float32, (3,), "target")
        req = nrc_request(NRC_REQ_TRAIN, enc.data_ptr(), target.data_ptr(), None, enc.shape[0])
        return self._submit(cache_id, req, (enc, target))

    def poll(self, ticket: int):
        """None while pending, else a dict with status, loss, skipped and timestamps."""
        res = nrc_result()
        rc = lib.nrc_serve_poll(self.handle, ticket, ctypes.byref(res))
        if rc == NRC_PENDING:
            return None
        self._live.pop(ticket, None)
        check(rc)
        return dict(status=res.status, loss=res.loss, skipped=res.skipped, t_submit=res.t_submit,
                    t_start=res.t_start, t_done=res.t_done)

    def drain(self):
        check(lib.nrc_serve_drain(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None and self.handle.value:
            check(lib.nrc_serve_drain(self.handle))
            check(lib.nrc_serve_destroy(self.handle))
            self.handle = None

    def __del__(self, _finalizing=sys.is_finalizing):
        if _finalizing() or lib is None:
            return
        try:
            self.close()
        except Exception:
            pass
