"""Float64 Voice render, vectorised over voices (torch CPU, autograd-capable).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The Voice (Section 3.2) is a monophonic keyboard, six ADSR envelopes (two
general ones plus a rate and an amplitude ADSR per LFO), two LFOs, a
modulation mixer, a sine VCO, a square-saw VCO, a noise generator, VCAs and an
audio mixer.  Control modules (ADSR, LFO) run at the control rate (441 Hz by
default, Section 3.1); their outputs are upsampled to the audio rate before
the audio modules use them (Section 3.2).  Parameters are stored normalised in
[0, 1] and mapped to human-readable values through min, max, curve and
symmetry hyperparameters (Section 3.3).

The paper gives the module list and routing in prose only; the formulas below
are readings of that prose, each stated and cited at its function.  Parameter order p = 0..77:

  0 midi_f0, 1 note duration (s)
  2 + 5k   ADSR k in (adsr_1, adsr_2, lfo_1 rate, lfo_1 amp, lfo_2 rate, lfo_2 amp):
           attack (s), decay (s), sustain, release (s), curve exponent alpha
  32 + 8i  LFO i: rate (Hz), rate-modulation depth (Hz), initial phase (rad),
           shape weights sin, tri, saw, rsaw, square
  48 + 4o + i  modulation gain G[o][i], outputs o = (vco_1 pitch, vco_1 amp,
           vco_2 pitch, vco_2 amp, noise amp), inputs i = (adsr_1, adsr_2,
           lfo_1, lfo_2)
  68 vco_1 (sine): tuning (st), pitch-mod depth (st), initial phase (rad)
  71 vco_2 (square-saw): tuning, pitch-mod depth, initial phase, shape
  75 mixer levels: sine, square-saw, noise
"""
from __future__ import annotations

import math

import numpy as np
import torch

from . import philox

F64 = torch.float64
TWO_PI = 2.0 * math.pi
NUM_PARAMS = 78

ADSR_BASE = (2, 7, 12, 17, 22, 27)
LFO_BASE = (32, 40)
G_BASE = 48
VCO1_BASE = 68
VCO2_BASE = 71
MIX_BASE = 75


def _t(x) -> torch.Tensor:
    return x if isinstance(x, torch.Tensor) else torch.as_tensor(np.asarray(x), dtype=F64)


# ---------------------------------------------------------------------------
# Parameters (Section 3.3)
# ---------------------------------------------------------------------------
def pow01(x: torch.Tensor, e: torch.Tensor) -> torch.Tensor:
    """x ** e for x in [0, 1], e > 0, with 0 ** e = 0 and a finite autograd graph at 0."""
    pos = x > 0
    safe = torch.where(pos, x, torch.ones_like(x))
    return torch.where(pos, safe ** e, torch.zeros_like(x))


def map_params(u: torch.Tensor, table) -> torch.Tensor:
    """Normalised u in [0, 1] -> human-readable values (Section 3.3).

    Reading: the curve c warps u as u ** (1/c) (c = 1 linear, c < 1 emphasises
    the top of the range, c > 1 the bottom); a symmetric parameter is centred:
    d = 2u - 1 is warped as sign(d) |d| ** (1/c) and mapped onto [min, max] so
    that u = 1/2 lands on the midpoint.
    """
    tab = _t(table)
    lo, hi, c, sym = tab[:, 0], tab[:, 1], tab[:, 2], tab[:, 3] > 0.5
    e = 1.0 / c
    lin = torch.where(c == 1.0, u, pow01(u, e))
    v_ns = lo + (hi - lo) * lin
    d = 2.0 * u - 1.0
    ad = d.abs()
    wd = torch.where(c == 1.0, ad, pow01(ad, e))
    v_s = lo + (hi - lo) * (1.0 + torch.sign(d) * wd) / 2.0
    return torch.where(sym, v_s, v_ns)


# ---------------------------------------------------------------------------
# Control modules at the control rate (Section 3.1)
# ---------------------------------------------------------------------------
def ramp(j: torch.Tensor, start: torch.Tensor, length: torch.Tensor) -> torch.Tensor:
    """clamp((j - start) / length, 0, 1); a zero-length ramp is the step [j >= start]."""
    pos = length > 0
    safe_len = torch.where(pos, length, torch.ones_like(length))
    lin = torch.clamp((j - start) / safe_len, 0.0, 1.0)
    return torch.where(pos, lin, (j >= start).to(F64))


def adsr(j, attack, decay, sustain, release, alpha, note_off, rc):
    """ADSR envelope at control samples j (Sections 3.1-3.2, Figure "ADSR").

    Reading: product of an attack rise, a decay fall to the sustain level and a
    release fall starting at note-off, each ramp raised to the curve exponent
    alpha.  Durations are in seconds and become control samples A = a * rc,
    D = d * rc, R = r * rc, O = note_off * rc (not rounded):

      env(j) = ramp(j; 0, A)^alpha * (S + (1 - S) (1 - ramp(j; A, D))^alpha)
               * (1 - ramp(j; O, R))^alpha
    """
    A, D, R, O = attack * rc, decay * rc, release * rc, note_off * rc
    att = ramp(j, torch.zeros_like(A), A)
    dec = ramp(j, A, D)
    rel = ramp(j, O, R)
    return pow01(att, alpha) * (sustain + (1.0 - sustain) * pow01(1.0 - dec, alpha)) \
        * pow01(1.0 - rel, alpha)


def exclusive_cumsum(x: torch.Tensor) -> torch.Tensor:
    """s[n] = sum_{k < n} x[k] along the last axis (s[0] = 0)."""
    c = torch.cumsum(x, dim=-1)
    return torch.cat([torch.zeros_like(c[..., :1]), c[..., :-1]], dim=-1)


def lfo_shapes(ph: torch.Tensor) -> torch.Tensor:
    """Unipolar shapes in [0, 1] of the phase fraction ph in [0, 1):
    sine (1 + sin 2 pi ph) / 2, triangle 1 - |2 ph - 1|, saw ph, reverse saw
    1 - ph, square [ph < 1/2].  Returns [..., 5]."""
    return torch.stack([(1.0 + torch.sin(TWO_PI * ph)) / 2.0,
                        1.0 - (2.0 * ph - 1.0).abs(),
                        ph,
                        1.0 - ph,
                        (ph < 0.5).to(F64)], dim=-1)


def lfo(j, rate, depth, phase0, weights, env_rate, rc):
    """Rate-modulated LFO at control rate (Section 3.2: each LFO has a rate ADSR).

    f(j) = max(0, rate + depth * env_rate(j)) Hz;
    phase(j) = phase0 / 2 pi + sum_{k < j} f(k) / rc  (cycles);
    output = weighted mean of the five shapes (0 if all weights are 0).
    """
    f = torch.clamp(rate + depth * env_rate, min=0.0)
    th = phase0 / TWO_PI + exclusive_cumsum(f / rc)
    ph = th - torch.floor(th)
    s = lfo_shapes(ph)                                   # [B, J, 5]
    wsum = weights.sum(-1, keepdim=True)                 # [B, 1]
    num = (s * weights[:, None, :]).sum(-1)              # [B, J]
    safe = torch.where(wsum > 0, wsum, torch.ones_like(wsum))
    return torch.where(wsum > 0, num / safe, torch.zeros_like(num))


def controls(v: torch.Tensor, J: int, rc: float) -> dict:
    """All control-rate signals of a batch of voices: six envelopes, both LFOs
    (after their amplitude ADSR), and the five modulation-mixer outputs.

    Modulation mixer reading: y_o(j) = sum_i G[o,i] x_i(j) / max(1, sum_i G[o,i])
    with inputs x = (adsr_1, adsr_2, lfo_1', lfo_2'), so every output stays in [0, 1].
    """
    B = v.shape[0]
    j = torch.arange(J, dtype=F64)[None, :]
    note_off = v[:, 1:2]
    env = []
    for b in ADSR_BASE:
        env.append(adsr(j, v[:, b:b + 1], v[:, b + 1:b + 2], v[:, b + 2:b + 3],
                        v[:, b + 3:b + 4], v[:, b + 4:b + 5], note_off, rc))
    lfos = []
    for i, b in enumerate(LFO_BASE):
        raw = lfo(j, v[:, b:b + 1], v[:, b + 1:b + 2], v[:, b + 2:b + 3],
                  v[:, b + 3:b + 8], env[2 + 2 * i], rc)
        lfos.append(raw * env[3 + 2 * i])                # control-rate VCA (amp ADSR)
    x = torch.stack([env[0], env[1], lfos[0], lfos[1]], dim=1)   # [B, 4, J]
    G = v[:, G_BASE:G_BASE + 20].reshape(B, 5, 4)
    norm = torch.clamp(G.sum(-1, keepdim=True), min=1.0)        # [B, 5, 1]
    y = torch.einsum("boi,bij->boj", G, x) / norm
    return {"env": env, "lfo": lfos, "x": x, "y": y}


# ---------------------------------------------------------------------------
# Audio modules (Sections 3.1-3.2)
# ---------------------------------------------------------------------------
def upsample(y: torch.Tensor, N: int, q: int) -> torch.Tensor:
    """Control -> audio rate by linear interpolation, control sample j at audio
    sample j*q, holding the last control value: a(n) = (1-t) y(j0) + t y(j0+1)."""
    J = y.shape[-1]
    n = torch.arange(N)
    j0 = n // q
    t = (n - j0 * q).to(F64) / q
    j1 = torch.clamp(j0 + 1, max=J - 1)
    return (1.0 - t) * y[..., j0] + t * y[..., j1]


def midi_to_hz(m):
    """12-tone equal temperament, A4 = MIDI 69 = 440 Hz."""
    return 440.0 * torch.pow(2.0, (m - 69.0) / 12.0)


def vco_phase(midi_f0, tuning, depth, phase0, a_pitch, sr):
    """Phase in cycles: theta(n) = phase0 / 2 pi + sum_{k < n} f(k) / sr, with
    f(n) = min(sr / 2, hz(midi_f0 + tuning + depth * a_pitch(n)))."""
    m = midi_f0 + tuning + depth * a_pitch
    f = torch.clamp(midi_to_hz(m), max=sr / 2.0)
    return phase0 / TWO_PI + exclusive_cumsum(f / sr)


def frac(th):
    return th - torch.floor(th)


def sine_vco(theta):
    return torch.sin(TWO_PI * frac(theta))


def squaresaw_gain(midi_f0, tuning, depth, sr):
    """Waveshaper gain K = 12000 / (f_hi log10 f_hi), f_hi the highest pitch the
    VCO can reach (floored at MIDI 0, capped at sr / 2)."""
    m_hi = torch.clamp(midi_f0 + tuning + torch.clamp(depth, min=0.0), min=0.0)
    f_hi = torch.clamp(midi_to_hz(m_hi), max=sr / 2.0)
    return 12000.0 / (f_hi * torch.log10(f_hi))


def squaresaw_vco(theta, shape, K):
    """Square-saw: a tanh-waveshaped sine (square, K sets the edge steepness)
    times a (1 + s cos) factor that skews it towards a saw as shape s -> 1:
    x2 = (1 - s/2) tanh(K sin 2 pi theta) (1 + s cos 2 pi theta), |x2| <= 9/8."""
    ph = TWO_PI * frac(theta)
    return (1.0 - shape / 2.0) * torch.tanh(K * torch.sin(ph)) * (1.0 + shape * torch.cos(ph))


def noise_batch(noise_seed: int, voice_ids, N: int) -> torch.Tensor:
    return torch.stack([torch.from_numpy(philox.noise(noise_seed, int(g), N)) for g in voice_ids])


def render_uniform(u, voice_ids, N: int, table, sr: float = 44100.0, rc: float = 441.0,
                   noise_seed: int = 0, mix_mode: int = 0, return_parts: bool = False):
    """Render B voices of N samples each.  u: [B, 78] normalised parameters
    (float64 tensor; may require grad).  Returns audio [B, N] float64."""
    q = int(round(sr / rc))
    assert abs(q * rc - sr) < 1e-9 * sr, "sample rate must be an integer multiple of the control rate"
    u = _t(u)
    v = map_params(u, table)
    J = -(-N // q)
    ctl = controls(v, J, rc)
    a = upsample(ctl["y"], N, q)                          # [B, 5, N]
    midi = v[:, 0:1]
    th1 = vco_phase(midi, v[:, 68:69], v[:, 69:70], v[:, 70:71], a[:, 0], sr)
    th2 = vco_phase(midi, v[:, 71:72], v[:, 72:73], v[:, 73:74], a[:, 2], sr)
    x1 = sine_vco(th1)
    K = squaresaw_gain(midi, v[:, 71:72], v[:, 72:73], sr)
    x2 = squaresaw_vco(th2, v[:, 74:75], K)
    x3 = noise_batch(noise_seed, voice_ids, N)
    v1, v2, v3 = x1 * a[:, 1], x2 * a[:, 3], x3 * a[:, 4]   # VCAs
    y = v[:, 75:76] * v1 + v[:, 76:77] * v2 + v[:, 77:78] * v3
    if mix_mode == 1:
        peak = y.abs().amax(-1, keepdim=True)             # peak-normalise if clipping
        y = y / torch.clamp(peak, min=1.0)
    if return_parts:
        return y, {"v": v, "ctl": ctl, "a": a, "th1": th1, "th2": th2, "x1": x1, "x2": x2,
                   "x3": x3, "K": K}
    return y


def render(u, voice_ids, lengths, table, sr: float = 44100.0, rc: float = 441.0,
           noise_seed: int = 0, mix_mode: int = 0) -> torch.Tensor:
    """Ragged render: voice i has lengths[i] samples; returns the packed float64
    buffer of sum(lengths) samples (voice i at offset sum(lengths[:i]))."""
    u = _t(u)
    ids = np.asarray(voice_ids, dtype=np.uint64)
    lengths = np.asarray(lengths, dtype=np.int64)
    out = [None] * len(lengths)
    for N in np.unique(lengths):
        idx = np.nonzero(lengths == N)[0]
        y = render_uniform(u[idx], ids[idx], int(N), table, sr, rc, noise_seed, mix_mode)
        for k, i in enumerate(idx):
            out[i] = y[k]
    return torch.cat(out) if out else torch.zeros(0, dtype=F64)


def silence_start(u, table, rc: float = 441.0) -> np.ndarray:
    """First control index after which every envelope is exactly 0 (end of the
    longest release), per voice; used by tests of the silent tail."""
    v = map_params(_t(u), table)
    ends = [v[:, 1] * rc + v[:, b + 3] * rc for b in ADSR_BASE]
    return torch.stack(ends, -1).amax(-1).detach().numpy()


def is_test(g: int) -> bool:
    """Train/test split: 9 * 1024 train voices, then 1024 test voices, repeating (Section 2.2)."""
    return (int(g) // 1024) % 10 == 9
