"""Four-operator FM voice (float64, torch CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Sections 3.2 and 7 announce a 4-operator FM architecture without describing
it.  Reading taken here: four sine operators on the keyboard's pitch, each
with a frequency ratio, a detune, an output level and its own ADSR (the
Voice's envelope, Section 3.1, at the control rate and upsampled linearly
as the Voice's control signals are); operator j modulates the phase of
operator i < j with index M[i][j] (in cycles), which covers every
feed-forward 4-operator routing ("algorithm"); the output is the mix of the
operators with weights w, divided by max(1, sum w).  Operators have no
self-feedback (it would make every sample depend on the previous one).

Parameters p = 0..43 (normalised u in [0, 1], mapped through a nebula
table exactly as the Voice's, Section 3.3):

  0 midi_f0, 1 note duration (s)
  2 + 8i   operator i = 0..3: ratio, detune (cents), level, attack (s),
           decay (s), sustain, release (s), envelope curve exponent alpha
  34..39   modulation indices M[0][1], M[0][2], M[0][3], M[1][2], M[1][3], M[2][3]
  40..43   mix weights w0..w3

Signal, sample n, operator frequency f_i = 440 2^((midi_f0 - 69) / 12)
ratio_i 2^(detune_i / 1200) (at most sr / 2), theta_i(n) = n f_i / sr:

  o_i(n) = level_i env_i(n) sin(2 pi (theta_i(n) + sum_{j > i} M[i][j] o_j(n)))

evaluated for i = 3, 2, 1, 0, and y(n) = sum_i w_i o_i(n) / max(1, sum_i w_i).
"""
from __future__ import annotations


import numpy as np
import torch

from . import philox
from .voice import TWO_PI, adsr, map_params, upsample

F64 = torch.float64
NUM_PARAMS = 44
ARCH_TAG = 1                      # the parameter draw's architecture tag
OP_BASE = (2, 10, 18, 26)
MOD_BASE = 34
MIX_BASE = 40
PAIRS = ((0, 1), (0, 2), (0, 3), (1, 2), (1, 3), (2, 3))


def param_names() -> list[str]:
    names = ["keyboard.midi_f0", "keyboard.duration"]
    for i in range(4):
        names += [f"op_{i}.{f}" for f in ("ratio", "detune", "level", "attack", "decay",
                                          "sustain", "release", "alpha")]
    names += [f"mod.{i}<-{j}" for i, j in PAIRS]
    names += [f"mix.w{i}" for i in range(4)]
    assert len(names) == NUM_PARAMS
    return names


def sample_params(seed: int, voice_ids) -> np.ndarray:
    """The FM voice's normalised parameters: the counter-based draw with the
    architecture tag ARCH_TAG."""
    return philox.sample_params(seed, voice_ids, NUM_PARAMS, tag=ARCH_TAG)


def op_freq(v: torch.Tensor, i: int, sr: float) -> torch.Tensor:
    b = OP_BASE[i]
    f = 440.0 * torch.pow(torch.tensor(2.0, dtype=F64), (v[:, 0:1] - 69.0) / 12.0) * v[:, b:b + 1] \
        * torch.pow(torch.tensor(2.0, dtype=F64), v[:, b + 1:b + 2] / 1200.0)
    return torch.clamp(f, max=sr / 2.0)


def render_uniform(u, N: int, table, sr: float = 44100.0, rc: float = 441.0,
                   return_parts: bool = False) -> torch.Tensor:
    """B FM voices of N samples from normalised parameters u [B, 44]."""
    q = int(round(sr / rc))
    assert abs(q * rc - sr) < 1e-9 * sr
    u = u if isinstance(u, torch.Tensor) else torch.as_tensor(np.asarray(u), dtype=F64)
    v = map_params(u.to(F64), table)
    J = -(-N // q)
    j = torch.arange(J, dtype=F64)[None, :]
    n = torch.arange(N, dtype=F64)[None, :]
    note_off = v[:, 1:2]
    o = [None] * 4
    for i in (3, 2, 1, 0):
        b = OP_BASE[i]
        env = adsr(j, v[:, b + 3:b + 4], v[:, b + 4:b + 5], v[:, b + 5:b + 6], v[:, b + 6:b + 7],
                   v[:, b + 7:b + 8], note_off, rc)
        a = upsample(env, N, q)
        theta = n * op_freq(v, i, sr) / sr
        for k, (ii, jj) in enumerate(PAIRS):
            if ii == i:
                theta = theta + v[:, MOD_BASE + k:MOD_BASE + k + 1] * o[jj]
        o[i] = v[:, b + 2:b + 3] * a * torch.sin(TWO_PI * theta)
    w = v[:, MIX_BASE:MIX_BASE + 4]
    y = sum(w[:, i:i + 1] * o[i] for i in range(4)) / torch.clamp(w.sum(-1, keepdim=True), min=1.0)
    if return_parts:
        return y, {"v": v, "o": o}
    return y


def render(u, lengths, table, sr: float = 44100.0, rc: float = 441.0) -> torch.Tensor:
    """Ragged render: voice i has lengths[i] samples; the packed float64 buffer."""
    u = u if isinstance(u, torch.Tensor) else torch.as_tensor(np.asarray(u), dtype=F64)
    lengths = np.asarray(lengths, dtype=np.int64)
    out = [None] * len(lengths)
    for N in np.unique(lengths):
        idx = np.nonzero(lengths == N)[0]
        if N == 0:
            for i in idx:
                out[i] = torch.zeros(0, dtype=F64)
            continue
        y = render_uniform(u[idx], int(N), table, sr, rc)
        for k, i in enumerate(idx):
            out[i] = y[k]
    return torch.cat(out) if out else torch.zeros(0, dtype=F64)
