"""Resonant low-pass filter module (a subtractive filter, Section 7's list of
modules to add) and its adjoint, on rendered voices.

Per voice: a base cutoff (MIDI note number), a modulation depth (semitones
per unit of a control-rate signal env, one value per control period) and
the resonance Q; each control period runs the cookbook second-order
low-pass at its cutoff as a direct-form-I recurrence (see synth.h).
Argument marshalling only: the filter and its adjoint run in libsynth.so's
kernels.  ``LowPass`` is the autograd function (gradients to the input
audio, the per-voice parameters and env).
"""
from __future__ import annotations

import ctypes

import torch

from . import _dev_ptr, _native, _stream

F32 = torch.float32
F64 = torch.float64


def _sig(L):
    vp, i64, i32, f64 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_double
    L.synth_vcf_state_chunks.restype = i64
    L.synth_vcf_state_chunks.argtypes = [i64, i32]
    L.synth_vcf_lowpass.restype = ctypes.c_int
    L.synth_vcf_lowpass.argtypes = [vp, vp, i64, i64, i64, vp, i64, vp, i32, f64, vp, vp, i64, vp,
                                    vp]
    L.synth_vcf_lowpass_backward.restype = ctypes.c_int
    L.synth_vcf_lowpass_backward.argtypes = [vp, vp, vp, i64, i64, i64, vp, i64, vp, i32, f64, vp,
                                             i64, vp, vp, vp, vp, vp]
    return L


_L = None


def lib():
    global _L
    if _L is None:
        _L = _sig(_native.lib())
    return _L


def _shape(x, offsets, max_samples):
    if offsets is None:
        if x.dim() != 2:
            raise ValueError("uniform audio must be [batch, n_samples]")
        return x.shape[0], x.shape[1], x.shape[1]
    B = offsets.numel() - 1
    if max_samples is None:
        max_samples = int(torch.diff(offsets).max().item()) if B > 0 else 1
    return B, 0, int(max_samples)


def state_chunks(max_samples: int, period: int = 100) -> int:
    return int(lib().synth_vcf_state_chunks(int(max_samples), int(period)))


def lowpass(x: torch.Tensor, env: torch.Tensor, params: torch.Tensor, period: int = 100,
            sample_rate: float = 44100.0, offsets: torch.Tensor | None = None,
            max_samples: int | None = None, keep_states: bool = False, out=None,
            order: torch.Tensor | None = None):
    """Filter voices: x [B, N] (or packed with offsets), env [B, >= ceil(len /
    period)] float32, params [B, 3] float32 (cutoff, depth, Q).  Returns y
    (and the chunk states the backward pass needs, with keep_states).
    `order` (int32 [B], a permutation) is the order in which workgroups take
    the voices; results do not depend on it."""
    B, N, lmax = _shape(x, offsets, max_samples)
    if out is None:
        out = torch.empty_like(x)
    states, sld = None, 0
    if keep_states and B > 0:
        sld = state_chunks(lmax, period)
        states = torch.empty(B, sld, 2, dtype=F64, device=x.device)
    if B > 0:
        _native.check("synth_vcf_lowpass", lib().synth_vcf_lowpass(
            _dev_ptr(x, "x", F32), _dev_ptr(offsets, "offsets", torch.int64, B + 1) if offsets is not None else None,
            B, N, lmax, _dev_ptr(env, "env", F32), env.stride(0), _dev_ptr(params, "params", F32, 3 * B),
            int(period), float(sample_rate), _dev_ptr(out, "y", F32),
            states.data_ptr() if states is not None else None, sld,
            _dev_ptr(order, "order", torch.int32, B) if order is not None else None, _stream(x.device)))
    return (out, states) if keep_states else out


def lowpass_backward(x, grad_y, env, params, states, period: int = 100,
                     sample_rate: float = 44100.0, offsets=None, max_samples=None,
                     grad_env: bool = True, order: torch.Tensor | None = None):
    """(dL/dx, dL/dparams [B, 3], dL/denv or None) for the forward call that
    wrote `states` on the same inputs; `order` as for lowpass."""
    B, N, lmax = _shape(x, offsets, max_samples)
    gx = torch.empty_like(x)
    gp = torch.empty(B, 3, dtype=F32, device=x.device)
    ge = torch.zeros_like(env) if grad_env else None
    if B > 0:
        _native.check("synth_vcf_lowpass_backward", lib().synth_vcf_lowpass_backward(
            _dev_ptr(x, "x", F32), _dev_ptr(grad_y, "grad_y", F32, x.numel()),
            _dev_ptr(offsets, "offsets", torch.int64, B + 1) if offsets is not None else None,
            B, N, lmax, _dev_ptr(env, "env", F32), env.stride(0), _dev_ptr(params, "params", F32, 3 * B),
            int(period), float(sample_rate), _dev_ptr(states, "states", F64), states.shape[1],
            _dev_ptr(gx, "grad_x", F32), _dev_ptr(gp, "grad_params", F32),
            _dev_ptr(ge, "grad_env", F32) if ge is not None else None,
            _dev_ptr(order, "order", torch.int32, B) if order is not None else None, _stream(x.device)))
    return gx, gp, ge


class LowPass(torch.autograd.Function):
    """y = lowpass(x, env, params) on uniform [B, N] audio, differentiable in
    x, env and params."""

    @staticmethod
    def forward(ctx, x, env, params, period=100, sample_rate=44100.0):
        x, env, params = x.contiguous().float(), env.contiguous().float(), params.contiguous().float()
        y, states = lowpass(x, env, params, period, sample_rate, keep_states=True)
        ctx.save_for_backward(x, env, params, states)
        ctx.cfg = (period, sample_rate)
        return y

    @staticmethod
    def backward(ctx, gy):
        x, env, params, states = ctx.saved_tensors
        period, sr = ctx.cfg
        gx, gp, ge = lowpass_backward(x, gy.contiguous().float(), env, params, states, period, sr)
        return gx, ge, gp, None, None
