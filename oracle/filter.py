"""Resonant low-pass filter module (float64, torch CPU, autograd-capable).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 7 of the paper lists subtractive filters among the modules to add.
Reading taken here (the paper gives no formulas): a voltage-controlled
resonant low-pass filter, the second-order low-pass section of R.
Bristow-Johnson's "Audio EQ Cookbook", whose cutoff is driven by a
control-rate signal env[j] (for instance an ADSR) one control period at a
time.  Per voice: a base cutoff as a MIDI note number, a modulation depth in
semitones and the resonance Q.  Control period j (samples [j q, (j + 1) q))
uses

    f_j   = clamp(440 * 2 ** ((cutoff + depth * env[j] - 69) / 12), F_MIN, F_MAX * sr)
    w_j   = 2 pi f_j / sr,   c = cos w_j,   s = sin w_j,   alpha = s / (2 Q)
    b0 = b2 = (1 - c) / 2 / (1 + alpha),   b1 = (1 - c) / (1 + alpha)
    a1 = -2 c / (1 + alpha),               a2 = (1 - alpha) / (1 + alpha)

and the direct-form-I recurrence (zero initial state, coefficients switched
at period boundaries, the input and output histories carried across them)

    y[n] = b0 x[n] + b1 x[n-1] + b2 x[n-2] - a1 y[n-1] - a2 y[n-2].

The section has unit gain at DC, a zero at Nyquist and gain Q at the cutoff.
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64
F_MIN = 10.0          # Hz
F_MAX = 0.45          # fraction of the sample rate


def _t(x) -> torch.Tensor:
    """float64 tensor view of x (tensors keep their autograd graph)."""
    if isinstance(x, torch.Tensor):
        return x if x.dtype == F64 else x.to(F64)
    return torch.as_tensor(np.asarray(x), dtype=F64)


def cutoff_hz(cutoff, depth, env, sr: float) -> torch.Tensor:
    """f[b, j] from the base cutoff (MIDI note), depth (semitones) and env [B, J]."""
    m = _t(cutoff)[:, None] + _t(depth)[:, None] * _t(env)
    f = 440.0 * torch.pow(torch.tensor(2.0, dtype=F64), (m - 69.0) / 12.0)
    return torch.clamp(f, F_MIN, F_MAX * sr)


def coefficients(f, q, sr: float):
    """(b0, b1, b2, a1, a2) of the cookbook low-pass at cutoff f [B, J] Hz and Q [B]."""
    w = 2.0 * math.pi * _t(f) / sr
    c, s = torch.cos(w), torch.sin(w)
    alpha = s / (2.0 * _t(q)[:, None])
    a0 = 1.0 + alpha
    b0 = (1.0 - c) / 2.0 / a0
    b1 = (1.0 - c) / a0
    a1 = -2.0 * c / a0
    a2 = (1.0 - alpha) / a0
    return b0, b1, b0, a1, a2


def lowpass(x, env, cutoff, depth, q, period: int, sr: float = 44100.0) -> torch.Tensor:
    """y [B, N] for x [B, N], env [B, J] with J >= ceil(N / period)."""
    x = _t(x)
    B, N = x.shape
    b0, b1, b2, a1, a2 = coefficients(cutoff_hz(cutoff, depth, env, sr), q, sr)
    zero = torch.zeros(B, dtype=F64)
    x1 = x2 = y1 = y2 = zero
    out = []
    for n in range(N):
        j = n // period
        xn = x[:, n]
        yn = b0[:, j] * xn + b1[:, j] * x1 + b2[:, j] * x2 - a1[:, j] * y1 - a2[:, j] * y2
        out.append(yn)
        x2, x1 = x1, xn
        y2, y1 = y1, yn
    return torch.stack(out, dim=1) if out else x.new_zeros(B, 0)


def lowpass_ragged(x_list, env, cutoff, depth, q, period: int, sr: float = 44100.0):
    """The filter on voices of different lengths (a list of 1-D arrays)."""
    return [lowpass(_t(x)[None, :], _t(env)[b:b + 1], _t(cutoff)[b:b + 1], _t(depth)[b:b + 1],
                    _t(q)[b:b + 1], period, sr)[0] for b, x in enumerate(x_list)]
