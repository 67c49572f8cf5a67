"""Four-operator FM voice (the FM architecture Sections 3.2 and 7 announce):
parameter draw and render (see synth.h for the parameter order and the
signal).  Argument marshalling only: both run in libsynth.so's kernels."""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _dev_ptr, _native, _stream

NUM_PARAMS = 44


class FmConfig(ctypes.Structure):
    _fields_ = [("sample_rate", ctypes.c_double),
                ("control_rate", ctypes.c_double),
                ("nebula", ctypes.POINTER(ctypes.c_double))]


def _sig(L):
    vp, i64, u64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64
    L.synth_fm_sample_params.restype = ctypes.c_int
    L.synth_fm_sample_params.argtypes = [u64, u64, i64, vp, vp, vp]
    L.synth_fm_render.restype = ctypes.c_int
    L.synth_fm_render.argtypes = [ctypes.POINTER(FmConfig), vp, i64, vp, i64, vp, vp, vp]
    return L


_L = None


def lib():
    global _L
    if _L is None:
        _L = _sig(_native.lib())
    return _L


def fm_sample_params(seed: int, first_g: int = 0, batch: int | None = None,
                     voice_ids: torch.Tensor | None = None, device="cuda") -> torch.Tensor:
    """Normalised FM parameters [B, 44] float32 (the FM voice's draw stream)."""
    if voice_ids is not None:
        batch, device = voice_ids.numel(), voice_ids.device
    if batch is None:
        raise ValueError("batch or voice_ids is required")
    out = torch.empty(batch, NUM_PARAMS, dtype=torch.float32, device=device)
    _native.check("synth_fm_sample_params", lib().synth_fm_sample_params(
        int(seed) & (2 ** 64 - 1), int(first_g), int(batch),
        _dev_ptr(voice_ids, "voice_ids", torch.uint64, batch) if voice_ids is not None else None,
        out.data_ptr(), _stream(out.device)))
    return out


def fm_render(params: torch.Tensor, nebula, n_samples: int | None = None,
              offsets: torch.Tensor | None = None, sample_rate: float = 44100.0,
              control_rate: float = 441.0, out: torch.Tensor | None = None,
              order: torch.Tensor | None = None) -> torch.Tensor:
    """Render B FM voices: [B, n_samples], or the packed buffer with offsets.
    `order` (int32 [B], a permutation) is the order in which workgroups take
    the voices; results do not depend on it."""
    B = params.shape[0]
    tab = np.ascontiguousarray(np.asarray(nebula, dtype=np.float64).reshape(NUM_PARAMS, 4))
    cfg = FmConfig(float(sample_rate), float(control_rate),
                   tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    total = int(offsets[-1].item()) if offsets is not None and out is None else (
        out.numel() if out is not None else B * int(n_samples))
    if out is None:
        out = torch.empty(total, dtype=torch.float32, device=params.device)
    _native.check("synth_fm_render", lib().synth_fm_render(
        ctypes.byref(cfg), _dev_ptr(params, "params", torch.float32, B * NUM_PARAMS), B,
        _dev_ptr(offsets, "offsets", torch.int64, B + 1) if offsets is not None else None,
        int(n_samples) if offsets is None else 0, _dev_ptr(out, "audio", torch.float32, total),
        _dev_ptr(order, "order", torch.int32, B) if order is not None else None,
        _stream(params.device)))
    del tab
    if offsets is None:
        return out.view(B, int(n_samples))
    return out
