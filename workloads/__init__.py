"""Seeded, synthetic workload definitions shared by the oracle, the tests and the bench.

This module holds *inputs only*: the nebula tables (per-parameter range
hyperparameters), seeds, batch shapes and the ragged length recipe.  It
contains none of the voice's arithmetic; the parameter draw, the range
mapping and every signal stage are implemented separately by the oracle
(``oracle/``) and by the HIP library (``paper_2104_12922_amd/``).

Paper context (arXiv 2104.12922): a nebula is one choice of the per-parameter
hyperparameters min, max, curve and symmetry (Section 3.3); the default Voice
has 78 latent parameters (Section 1.1) and renders 4 s sounds at 44.1 kHz with
a 441 Hz control rate (Sections 2.2 and 3.1).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

NUM_PARAMS = 78
SAMPLE_RATE = 44100.0
CONTROL_RATE = 441.0

# Seeds of the synthetic workloads.
SEED_PARAM = 0
SEED_TARGET = 1
SEED_TRAIN = 10
SEED_HELDOUT = 11
SEED_MATCH = 20
SEED_RS = 21
SEED_CAND_NOISE = 22

_ADSR_NAMES = ("adsr_1", "adsr_2", "lfo_1_rate_adsr", "lfo_1_amp_adsr",
               "lfo_2_rate_adsr", "lfo_2_amp_adsr")
_ADSR_FIELDS = ("attack", "decay", "sustain", "release", "alpha")
_LFO_FIELDS = ("rate", "mod_depth", "initial_phase", "w_sin", "w_tri", "w_saw",
               "w_rsaw", "w_sqr")
MOD_OUTPUTS = ("vco_1_pitch", "vco_1_amp", "vco_2_pitch", "vco_2_amp", "noise_amp")
MOD_INPUTS = ("adsr_1", "adsr_2", "lfo_1", "lfo_2")


def param_names() -> list[str]:
    """Canonical parameter order p = 0..77 of the default Voice (Section 3.2)."""
    names = ["keyboard.midi_f0", "keyboard.duration"]
    for a in _ADSR_NAMES:
        names += [f"{a}.{f}" for f in _ADSR_FIELDS]
    for l in ("lfo_1", "lfo_2"):
        names += [f"{l}.{f}" for f in _LFO_FIELDS]
    for o in MOD_OUTPUTS:
        names += [f"mod_matrix.{o}<-{i}" for i in MOD_INPUTS]
    names += ["vco_1.tuning", "vco_1.mod_depth", "vco_1.initial_phase"]
    names += ["vco_2.tuning", "vco_2.mod_depth", "vco_2.initial_phase", "vco_2.shape"]
    names += ["mixer.level_sine", "mixer.level_squaresaw", "mixer.level_noise"]
    assert len(names) == NUM_PARAMS
    return names


@dataclass
class Nebula:
    """Per-parameter hyperparameters (Section 3.3): range [lo, hi], curve, symmetric flag."""
    lo: np.ndarray
    hi: np.ndarray
    curve: np.ndarray
    sym: np.ndarray  # bool
    name: str = "default"

    def table(self) -> np.ndarray:
        """[78, 4] float64 table (lo, hi, curve, sym) - the layout the C ABI takes."""
        return np.stack([self.lo, self.hi, self.curve, self.sym.astype(np.float64)], axis=1).copy()


def default_nebula(duration_min: float = 0.0) -> Nebula:
    """Default Voice nebula with the ranges of the 4 s plain-render workload.

    midi_f0 24..84, note duration 0..4 s (0.1..4 s for the ragged workload),
    ADSR attack/decay/release 0..2 s, sustain 0..1, curve exponent 0.1..6,
    LFO rate 0..20 Hz, pitch modulation +-12 semitones, all curves linear.
    """
    lo = np.zeros(NUM_PARAMS)
    hi = np.ones(NUM_PARAMS)
    curve = np.ones(NUM_PARAMS)
    sym = np.zeros(NUM_PARAMS, dtype=bool)
    lo[0], hi[0] = 24.0, 84.0
    lo[1], hi[1] = duration_min, 4.0
    for k in range(6):
        b = 2 + 5 * k
        lo[b:b + 5] = (0.0, 0.0, 0.0, 0.0, 0.1)
        hi[b:b + 5] = (2.0, 2.0, 1.0, 2.0, 6.0)
    for i in range(2):
        b = 32 + 8 * i
        lo[b:b + 3] = (0.0, -10.0, -math.pi)
        hi[b:b + 3] = (20.0, 20.0, math.pi)
    lo[68:71] = (-24.0, -12.0, -math.pi)
    hi[68:71] = (24.0, 12.0, math.pi)
    sym[68:70] = True
    lo[71:75] = (-24.0, -12.0, -math.pi, 0.0)
    hi[71:75] = (24.0, 12.0, math.pi, 1.0)
    sym[71:73] = True
    return Nebula(lo, hi, curve, sym, name="default" if duration_min == 0 else "default_ragged")


def curved_test_nebula() -> Nebula:
    """A nebula exercising non-linear curves and symmetric mappings (test input only)."""
    n = default_nebula()
    rng = np.random.default_rng(1234)
    n.curve = rng.choice([0.25, 0.5, 1.0, 2.0, 4.0], size=NUM_PARAMS)
    n.sym = n.sym.copy()
    n.sym[[32 + 1, 40 + 1]] = True  # LFO depths symmetric too
    n.name = "curved"
    return n


FM_NUM_PARAMS = 44


def fm_default_nebula(duration_min: float = 0.0) -> Nebula:
    """Default nebula of the 4-operator FM voice (parameter order in
    oracle/fm.py): midi_f0 24..84, note duration 0..4 s, operator ratio
    0.5..8 (curve 2: low ratios favoured), detune +-50 cents (symmetric),
    level 0..1, ADSR ranges as the Voice's, modulation index 0..2 cycles
    (curve 2), mix weights 0..1."""
    lo = np.zeros(FM_NUM_PARAMS)
    hi = np.ones(FM_NUM_PARAMS)
    curve = np.ones(FM_NUM_PARAMS)
    sym = np.zeros(FM_NUM_PARAMS, dtype=bool)
    lo[0], hi[0] = 24.0, 84.0
    lo[1], hi[1] = duration_min, 4.0
    for i in range(4):
        b = 2 + 8 * i
        lo[b:b + 8] = (0.5, -50.0, 0.0, 0.0, 0.0, 0.0, 0.0, 0.1)
        hi[b:b + 8] = (8.0, 50.0, 1.0, 2.0, 2.0, 1.0, 2.0, 6.0)
        curve[b] = 2.0
        sym[b + 1] = True
    hi[34:40] = 2.0
    curve[34:40] = 2.0
    return Nebula(lo, hi, curve, sym, name="fm_default" if duration_min == 0 else "fm_default_ragged")


# ----------------------------------------------------------------------------
# Workload shapes
# ----------------------------------------------------------------------------
@dataclass
class Workload:
    name: str
    batch: int
    seed: int
    first_g: int
    lengths: np.ndarray  # samples per voice, int64 [B]
    nebula: Nebula
    sample_rate: float = SAMPLE_RATE
    control_rate: float = CONTROL_RATE
    noise_seed: int | None = None
    extra: dict = field(default_factory=dict)

    @property
    def offsets(self) -> np.ndarray:
        o = np.zeros(self.batch + 1, dtype=np.int64)
        np.cumsum(self.lengths, out=o[1:])
        return o

    @property
    def total_samples(self) -> int:
        return int(self.lengths.sum())

    @property
    def uniform(self) -> bool:
        return bool((self.lengths == self.lengths[0]).all())

    def key_noise(self) -> int:
        return self.seed if self.noise_seed is None else self.noise_seed


def plain_render(batch: int = 128, seconds: float = 4.0, seed: int = SEED_PARAM) -> Workload:
    """Plain render: 128 voices x 4 s at 44.1 kHz, voice ids 0..B-1."""
    n = int(round(seconds * SAMPLE_RATE))
    return Workload("plain_render_b%d_%gs" % (batch, seconds), batch, seed, 0,
                    np.full(batch, n, dtype=np.int64), default_nebula())


def ragged_batch(batch: int = 16384, seed: int = SEED_PARAM) -> Workload:
    """Batched throughput workload: lengths (1, 2, 4) s by voice index mod 3,
    note durations uniform 0.1..4 s, packed back to back (ragged offsets)."""
    secs = np.array([1, 2, 4], dtype=np.int64)[np.arange(batch) % 3]
    lengths = secs * int(SAMPLE_RATE)
    return Workload("ragged_b%d_1-2-4s" % batch, batch, seed, 0, lengths,
                    default_nebula(duration_min=0.1))


def gradient_batch(batch: int = 256) -> Workload:
    return Workload("grad_b%d_4s" % batch, batch, SEED_PARAM, 0,
                    np.full(batch, int(4 * SAMPLE_RATE), dtype=np.int64), default_nebula())



def mlp_init(seed: int = 0, d_in: int = 8192, d_h: int = 1024, d_out: int = 78) -> dict:
    """Initial weights of the proposal MLP (inputs, drawn from a seeded numpy
    generator): He-normal hidden layers, a 1/sqrt(fan_in) output layer, zero
    biases.  Weights are stored transposed (K-major): w1t [d_h][d_in], etc."""
    rng = np.random.default_rng(seed)
    return {
        "w1t": (rng.standard_normal((d_h, d_in)) * math.sqrt(2.0 / d_in)).astype(np.float32),
        "b1": np.zeros(d_h, np.float32),
        "w2t": (rng.standard_normal((d_h, d_h)) * math.sqrt(2.0 / d_h)).astype(np.float32),
        "b2": np.zeros(d_h, np.float32),
        "w3t": (rng.standard_normal((d_out, d_h)) * math.sqrt(1.0 / d_h)).astype(np.float32),
        "b3": np.zeros(d_out, np.float32),
    }
