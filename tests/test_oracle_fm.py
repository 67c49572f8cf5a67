"""Pins of the 4-operator FM voice oracle (oracle/fm.py): a lone carrier is
a plain sine, two-operator FM matches its Bessel-series expansion (pinning
the index's unit and the modulation's direction), a silent modulator
leaves its carrier a sine, the mix normalisation, the frequency cap, the
shared envelope, and the parameter draw's architecture tag."""
import math

import numpy as np
import scipy.special
import torch

import workloads as W
from oracle import fm as FM
from oracle import philox

SR = 44100.0


def _table(**fix):
    """A nebula whose min = max pins each named parameter to a value."""
    t = W.fm_default_nebula().table()
    names = FM.param_names()
    for k, val in fix.items():
        p = names.index(k)
        t[p, 0] = t[p, 1] = val
        t[p, 2], t[p, 3] = 1.0, 0.0
    return t


def _steady(i, ratio=1.0, level=1.0, detune=0.0):
    """Operator i at a constant envelope of 1 (attack 0, sustain 1, no release)."""
    return {f"op_{i}.ratio": ratio, f"op_{i}.detune": detune, f"op_{i}.level": level,
            f"op_{i}.attack": 0.0, f"op_{i}.decay": 0.0, f"op_{i}.sustain": 1.0,
            f"op_{i}.release": 0.0, f"op_{i}.alpha": 1.0}


def _silent(i):
    return {f"op_{i}.level": 0.0}


def _base(**kw):
    d = {"keyboard.midi_f0": 69.0, "keyboard.duration": 10.0, "mix.w1": 0.0, "mix.w2": 0.0,
         "mix.w3": 0.0, "mix.w0": 1.0}
    for k in ("mod.0<-1", "mod.0<-2", "mod.0<-3", "mod.1<-2", "mod.1<-3", "mod.2<-3"):
        d[k] = 0.0
    for i in (1, 2, 3):
        d.update(_silent(i))
    d.update(_steady(0))
    d.update(kw)
    return d


def test_lone_carrier_is_a_sine():
    N = 3000
    u = np.random.default_rng(0).uniform(size=(2, FM.NUM_PARAMS))
    t = _table(**_base(**_steady(0, ratio=1.5, detune=12.0)))
    y = FM.render_uniform(torch.tensor(u), N, t).numpy()
    f = 440.0 * 1.5 * 2.0 ** (12.0 / 1200.0)
    ref = np.sin(2 * np.pi * f * np.arange(N) / SR)
    assert np.max(np.abs(y - ref[None])) < 1e-9


def test_two_operator_fm_is_its_bessel_series():
    # carrier 440 Hz, modulator ratio 0.25 (110 Hz), index beta = 0.4 cycles at level 0.75:
    # sin(2 pi (fc t + beta L sin(2 pi fm t))) = sum_k J_k(2 pi beta L) sin(2 pi (fc + k fm) t)
    N = 4000
    beta, L = 0.4, 0.75
    fix = _base(**_steady(1, ratio=0.25, level=L))
    fix["mod.0<-1"] = beta
    y = FM.render_uniform(torch.tensor(np.full((1, FM.NUM_PARAMS), 0.5)), N, _table(**fix)).numpy()[0]
    t = np.arange(N) / SR
    I = 2 * np.pi * beta * L
    ref = sum(scipy.special.jv(k, I) * np.sin(2 * np.pi * (440.0 + k * 110.0) * t) for k in range(-30, 31))
    assert np.max(np.abs(y - ref)) < 1e-9


def test_silent_modulator_and_routing_direction():
    N = 2000
    # operator 0 modulates nobody: giving it a large index on op 3's phase does nothing
    fix = _base(**_steady(3, ratio=2.0))
    fix["mix.w0"], fix["mix.w3"] = 0.0, 1.0
    fix["mod.0<-3"] = 1.7          # 3 modulates 0, not the other way round
    y = FM.render_uniform(torch.tensor(np.full((1, FM.NUM_PARAMS), 0.5)), N, _table(**fix)).numpy()[0]
    assert np.max(np.abs(y - np.sin(2 * np.pi * 880.0 * np.arange(N) / SR))) < 1e-9
    # a modulator at level 0 leaves its carrier a sine
    fix = _base(**_steady(2, ratio=3.0, level=0.0))
    fix["mod.0<-2"] = 2.0
    y = FM.render_uniform(torch.tensor(np.full((1, FM.NUM_PARAMS), 0.5)), N, _table(**fix)).numpy()[0]
    assert np.max(np.abs(y - np.sin(2 * np.pi * 440.0 * np.arange(N) / SR))) < 1e-9


def test_mix_normalisation_and_frequency_cap():
    N = 500
    fix = _base(**_steady(1, ratio=2.0), **{"mix.w1": 1.0, "mix.w0": 1.0})
    y = FM.render_uniform(torch.tensor(np.full((1, FM.NUM_PARAMS), 0.5)), N, _table(**fix)).numpy()[0]
    n = np.arange(N) / SR
    assert np.max(np.abs(y - (np.sin(2 * np.pi * 440 * n) + np.sin(2 * np.pi * 880 * n)) / 2)) < 1e-9
    fix = _base(**_steady(0, ratio=8.0), **{"keyboard.midi_f0": 127.0})
    v = torch.tensor(np.full((1, FM.NUM_PARAMS), 0.5))
    from oracle.voice import map_params
    f = FM.op_freq(map_params(v, _table(**fix)), 0, SR)
    assert float(f) == SR / 2


def test_envelope_is_the_voice_adsr():
    from oracle.voice import adsr, upsample
    N = 6000
    u = np.random.default_rng(4).uniform(size=(3, FM.NUM_PARAMS))
    t = W.fm_default_nebula().table()
    y, parts = FM.render_uniform(torch.tensor(u), N, t, return_parts=True)
    v = parts["v"]
    j = torch.arange(60, dtype=torch.float64)[None, :]
    b = FM.OP_BASE[3]                   # ratio, detune, level, attack, decay, sustain, release, alpha
    env = adsr(j, v[:, b + 3:b + 4], v[:, b + 4:b + 5], v[:, b + 5:b + 6], v[:, b + 6:b + 7],
               v[:, b + 7:b + 8], v[:, 1:2], 441.0)
    a = upsample(env, N, 100)
    lvl = v[:, b + 2:b + 3]
    ref = lvl * a * torch.sin(2 * math.pi * torch.arange(N, dtype=torch.float64)[None] * FM.op_freq(v, 3, SR) / SR)
    assert torch.max(torch.abs(parts["o"][3] - ref)) < 1e-12


def test_parameter_draw_tag():
    ids = np.array([0, 5, 2 ** 40 + 3], dtype=np.uint64)
    a = FM.sample_params(7, ids)
    b = philox.sample_params(7, ids, FM.NUM_PARAMS)          # tag 0: the Voice's stream
    assert a.shape == (3, 44) and not np.array_equal(a, b)
    # brute force: counter (g lo, g hi, block, 1), key = seed
    for r, g in enumerate(ids):
        for blk in range(11):
            ctr = np.array([[int(g) & 0xFFFFFFFF, int(g) >> 32, blk, 1]], dtype=np.uint64)
            w = philox.philox4x32(ctr, np.array([7, 0], dtype=np.uint64))[0]
            assert np.array_equal(a[r, 4 * blk:4 * blk + 4], philox.u24(w))
