"""Pins of the float64 voice oracle against closed forms, invariants and brute force.

Each test checks the oracle against something other than itself: a textbook
closed form (piecewise-linear ADSR, constant-pitch sine, geometric phase sum),
an invariant (superposition, half-wave symmetry, weight scaling), or the
scalar loop-by-loop implementation on tiny inputs.
"""
import math

import numpy as np
import pytest
import torch

import workloads as W
from oracle import brute, philox, voice

F64 = torch.float64
SR, RC = 44100.0, 441.0


def u_for(values: dict, base_u=None, table=None):
    """Normalised parameter row that maps to the given human-readable values
    (default nebula: every curve is linear, so u = (v - lo) / (hi - lo))."""
    tab = W.default_nebula().table() if table is None else table
    u = np.full(78, 0.5) if base_u is None else np.array(base_u, dtype=np.float64)
    for p, val in values.items():
        lo, hi = tab[p, 0], tab[p, 1]
        u[p] = (val - lo) / (hi - lo)
    return u


def silent_matrix():
    return {48 + k: 0.0 for k in range(20)}


# ---------------------------------------------------------------------------
# Parameter mapping
# ---------------------------------------------------------------------------
def test_map_linear_endpoints_and_midpoint(nebula_table):
    tab = nebula_table
    u = torch.tensor(np.stack([np.zeros(78), np.full(78, 0.5), np.full(78, 0.25)]), dtype=F64)
    v = voice.map_params(u, tab).numpy()
    assert np.array_equal(v[0], tab[:, 0])
    assert np.allclose(v[1], (tab[:, 0] + tab[:, 1]) / 2, rtol=0, atol=1e-15)
    assert np.allclose(v[2], tab[:, 0] + 0.25 * (tab[:, 1] - tab[:, 0]), rtol=0, atol=1e-14)


def test_map_curves_closed_form():
    tab = W.default_nebula().table()
    tab[:, 2] = 4.0
    tab[:, 3] = 0.0
    tab[5, 3] = 1.0
    u = torch.tensor([[0.3] * 78, [0.8] * 78], dtype=F64)
    v = voice.map_params(u, tab).numpy()
    lo, hi = tab[:, 0], tab[:, 1]
    assert np.allclose(v[0, 0], lo[0] + (hi[0] - lo[0]) * 0.3 ** 0.25, rtol=1e-15)
    # symmetric: d = 2u - 1 = -0.4 -> (1 - 0.4^(1/4)) / 2
    assert np.allclose(v[0, 5], lo[5] + (hi[5] - lo[5]) * (1 - 0.4 ** 0.25) / 2, rtol=1e-15)
    # odd symmetry about the midpoint and monotonicity
    us = torch.linspace(0, 1, 101, dtype=F64)[:, None].repeat(1, 78)
    vs = voice.map_params(us, tab).numpy()
    mid = (lo[5] + hi[5]) / 2
    assert np.allclose(vs[:, 5] - mid, -(vs[::-1, 5] - mid), atol=1e-14)
    assert (np.diff(vs, axis=0) >= 0).all()


# ---------------------------------------------------------------------------
# ADSR
# ---------------------------------------------------------------------------
def textbook_adsr(j, A, D, S, O, R):
    """Classic linear ADSR (alpha = 1) for O >= A + D: rise, fall to S, hold, release."""
    if j < A:
        return j / A
    if j < A + D:
        return 1 - (1 - S) * (j - A) / D
    if j < O:
        return S
    if j < O + R:
        return S * (1 - (j - O) / R)
    return 0.0


def _env(j, a, d, s, r, alpha, off, rc=RC):
    t = lambda x: torch.tensor([[x]], dtype=F64)
    return voice.adsr(torch.as_tensor(j, dtype=F64)[None, :], t(a), t(d), t(s), t(r), t(alpha),
                      t(off), rc)[0].numpy()


def test_adsr_linear_matches_textbook():
    rc = 100.0  # control samples per second: A = 20, D = 30, O = 100, R = 50
    j = np.arange(0, 200, dtype=np.float64)
    got = _env(j, 0.2, 0.3, 0.4, 0.5, 1.0, 1.0, rc)
    exp = np.array([textbook_adsr(x, 20, 30, 0.4, 100, 50) for x in j])
    assert np.allclose(got, exp, rtol=0, atol=1e-15)
    assert got[0] == 0.0 and got[20] == 1.0 and got[150:].max() == 0.0
    assert (got[50:100] == 0.4).all()


def test_adsr_curve_exponent_and_early_release():
    rc = 100.0
    j = np.arange(0, 120, dtype=np.float64)
    a2 = _env(j, 0.4, 0.2, 0.5, 0.3, 2.0, 0.25, rc)  # A=40, D=20, O=25, R=30
    for x in (5, 10, 24):
        assert math.isclose(a2[x], (x / 40) ** 2, rel_tol=1e-14)
    for x in (30, 39, 50):  # release during attack: multiplicative law
        exp = (min(x / 40, 1)) ** 2 * (0.5 + 0.5 * (1 - min(max((x - 40) / 20, 0), 1)) ** 2) \
            * (1 - min((x - 25) / 30, 1)) ** 2
        assert math.isclose(a2[x], exp, rel_tol=1e-14)
    assert a2[55:].max() == 0.0


def test_adsr_zero_lengths_are_steps():
    j = np.arange(0, 50, dtype=np.float64)
    e = _env(j, 0.0, 0.0, 0.7, 0.0, 3.0, 0.2, 100.0)  # O = 20
    assert (e[:20] == 0.7).all() and (e[20:] == 0.0).all()


# ---------------------------------------------------------------------------
# LFO
# ---------------------------------------------------------------------------
def _lfo(rate, depth, ph0, w, env_rate, J, rc=RC):
    t = lambda x: torch.tensor([[x]], dtype=F64)
    j = torch.arange(J, dtype=F64)[None, :]
    return voice.lfo(j, t(rate), t(depth), t(ph0), torch.tensor([w], dtype=F64),
                     torch.as_tensor(env_rate, dtype=F64)[None, :], rc)[0].numpy()


def test_lfo_pure_shapes_closed_form():
    J, rate, ph0 = 1764, 3.7, 1.1
    jj = np.arange(J)
    ph = (ph0 / (2 * np.pi) + rate * jj / RC) % 1.0
    zero = np.zeros(J)
    saw = _lfo(rate, 5.0, ph0, [0, 0, 1, 0, 0], zero, J)
    d = saw - ph
    assert np.abs(d - np.round(d)).max() < 1e-11        # equal modulo the saw's wrap
    sine = _lfo(rate, 0.0, ph0, [2, 0, 0, 0, 0], zero, J)
    assert np.allclose(sine, (1 + np.sin(ph0 + 2 * np.pi * rate * jj / RC)) / 2, atol=1e-11)
    tri = _lfo(rate, 0.0, ph0, [0, 1, 0, 0, 0], zero, J)
    assert np.allclose(tri, 1 - np.abs(2 * ph - 1), atol=1e-11)
    rs = _lfo(rate, 0.0, ph0, [0, 0, 0, 1, 0], zero, J)
    assert np.allclose(rs, 1 - ph, atol=1e-11)


def test_lfo_square_duty_and_weight_scaling():
    J = 64 * 40
    # rate 441/64 Hz: the phase step 1/64 is exact in binary, period 64 control samples
    sq = _lfo(441.0 / 64, 0.0, 0.0, [0, 0, 0, 0, 1], np.zeros(J), J)
    assert set(np.unique(sq)) == {0.0, 1.0}
    assert abs(sq.mean() - 0.5) < 1e-12
    assert (sq[:32] == 1).all() and (sq[32:64] == 0).all()
    w = [0.3, 0.1, 0.7, 0.2, 0.5]
    a = _lfo(2.0, 3.0, 0.4, w, np.linspace(0, 1, 500), 500)
    b = _lfo(2.0, 3.0, 0.4, [5 * x for x in w], np.linspace(0, 1, 500), 500)
    assert np.allclose(a, b, atol=1e-15)
    assert (_lfo(2.0, 0, 0, [0] * 5, np.zeros(10), 10) == 0).all()


def test_lfo_rate_modulation_and_clamp():
    J = 900
    env = np.ones(J)
    x = _lfo(2.0, 3.0, 0.0, [0, 0, 1, 0, 0], env, J)   # f = 5 Hz
    d = x - (5.0 * np.arange(J) / RC) % 1.0
    assert np.abs(d - np.round(d)).max() < 1e-11        # equal modulo the saw's wrap
    frozen = _lfo(2.0, -9.0, 0.6, [0, 0, 1, 0, 0], env, J)  # f = max(0, -7) = 0
    assert np.allclose(frozen, 0.6 / (2 * np.pi), atol=1e-15)


# ---------------------------------------------------------------------------
# Modulation mixer and upsampling
# ---------------------------------------------------------------------------
def test_mod_mixer_selects_and_normalises(nebula_table):
    u = philox.sample_params(0, np.arange(3))
    v = voice.map_params(torch.tensor(u), nebula_table)
    G = torch.zeros(3, 20, dtype=F64)
    G[:, 0 * 4 + 2] = 1.0                      # vco1 pitch <- lfo_1
    G[:, 1 * 4 + 0] = 0.25                     # vco1 amp <- adsr_1 (sum <= 1: plain)
    G[:, 1 * 4 + 1] = 0.5
    G[:, 2 * 4 + 0] = 2.0                      # gains sum to 4 -> divided by 4
    G[:, 2 * 4 + 3] = 2.0
    v[:, 48:68] = G
    c = voice.controls(v, 300, RC)
    x, y = c["x"], c["y"]
    assert torch.equal(y[:, 0], x[:, 2])
    assert torch.allclose(y[:, 1], 0.25 * x[:, 0] + 0.5 * x[:, 1], atol=1e-16)
    assert torch.allclose(y[:, 2], (x[:, 0] + x[:, 3]) / 2, atol=1e-16)
    assert (y[:, 3:] == 0).all()


def test_upsample_exact_at_control_points_and_linear():
    J, q = 20, 100
    y = torch.tensor(np.random.default_rng(1).random((2, J)))
    a = voice.upsample(y, J * q, q)
    assert torch.equal(a[:, ::q], y)
    lin = torch.arange(J, dtype=F64)[None, :] * 0.37 + 1.0
    al = voice.upsample(lin, (J - 1) * q, q)
    assert torch.allclose(al, 1.0 + 0.37 * torch.arange((J - 1) * q, dtype=F64) / q, atol=1e-14)
    tail = voice.upsample(y, J * q, q)[:, (J - 1) * q:]
    assert torch.allclose(tail, y[:, -1:].expand_as(tail), rtol=0, atol=1e-15)


# ---------------------------------------------------------------------------
# VCOs
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("midi", [24.0, 57.3, 69.0, 96.0, 120.0])
def test_constant_pitch_sine_closed_form(midi):
    N = 176400
    a = torch.zeros(1, N, dtype=F64)
    ph0 = 0.7
    th = voice.vco_phase(torch.tensor([[midi]], dtype=F64), 0.0, 5.0, ph0, a, SR)
    x = voice.sine_vco(th)[0].numpy()
    f = 440.0 * 2 ** ((midi - 69) / 12)
    n = np.arange(N)
    exp = np.sin(2 * np.pi * ((f / SR * n) % 1.0) + ph0)
    # float64 running sum of N increments: drift <= N * eps/2 * theta_max cycles
    bound = 2 * np.pi * N * 2.0 ** -53 * (f * N / SR) + 1e-12
    assert np.abs(x - exp).max() < bound


def test_linear_pitch_glide_is_geometric_sum():
    # pitch rises linearly by 3 semitones over one 100-sample segment
    q, N = 100, 100
    y = torch.tensor([[0.0, 1.0]], dtype=F64)
    a = voice.upsample(y, N, q)
    th = voice.vco_phase(torch.tensor([[60.0]], dtype=F64), 0.0, 3.0, 0.0, a, SR)[0].numpy()
    f0 = 440 * 2 ** ((60 - 69) / 12) / SR
    r = 2 ** (3.0 / 1200)
    k = np.arange(N)
    assert np.allclose(th, f0 * (r ** k - 1) / (r - 1), rtol=1e-12, atol=1e-15)
    # and against a brute-force double loop
    bf = [sum(440 * 2 ** ((60 + 3 * (i / 100) - 69) / 12) / SR for i in range(n)) for n in range(N)]
    assert np.allclose(th, bf, rtol=1e-13, atol=1e-15)


def test_squaresaw_gain_closed_form():
    K = voice.squaresaw_gain(torch.tensor([69.0, 0.0], dtype=F64), torch.tensor([0.0, -20.0], dtype=F64),
                             torch.tensor([-3.0, 5.0], dtype=F64), SR)
    assert math.isclose(float(K[0]), 12000 / (440 * math.log10(440)), rel_tol=1e-14)
    f_hi = 440 * 2 ** ((0 - 69) / 12)      # floored at MIDI 0
    assert math.isclose(float(K[1]), 12000 / (f_hi * math.log10(f_hi)), rel_tol=1e-14)


def test_squaresaw_symmetry_bound_and_square_limit():
    th = torch.linspace(0, 3, 30001, dtype=F64)
    for K in (0.5, 10.0, 1600.0):
        x0 = voice.squaresaw_vco(th, 0.0, K)
        xh = voice.squaresaw_vco(th + 0.5, 0.0, K)
        assert torch.allclose(x0, -xh, atol=1e-9)
        for s in (0.0, 0.3, 0.5, 1.0):
            assert voice.squaresaw_vco(th, s, K).abs().max() <= 9 / 8 + 1e-12
    sq = voice.squaresaw_vco(torch.tensor([0.1, 0.3, 0.6, 0.9], dtype=F64), 0.0, 1600.0)
    assert torch.allclose(sq, torch.tensor([1.0, 1.0, -1.0, -1.0], dtype=F64), atol=1e-12)
    # s = 1: (1/2) sign(sin)(1 + cos): one jump per period, from 0 at phase 1/2
    saw = voice.squaresaw_vco(th, 1.0, 1600.0)
    assert abs(float(saw[(th - 0.5).abs().argmin()])) < 1e-6


# ---------------------------------------------------------------------------
# Whole voice
# ---------------------------------------------------------------------------
def test_whole_voice_pure_sine_closed_form():
    vals = silent_matrix()
    vals.update({0: 60.0, 1: 4.0, 68: 3.0, 69: 7.0, 70: 0.5, 75: 0.8, 76: 0.0, 77: 0.0})
    vals.update({2: 0.0, 3: 0.0, 4: 1.0, 5: 0.0})      # adsr_1 = step to 1, held
    vals[48 + 4 * 1 + 0] = 1.0                        # vco1 amp <- adsr_1
    u = torch.tensor(u_for(vals))[None]
    N = 176400
    y = voice.render_uniform(u, [0], N, W.default_nebula().table(), noise_seed=0)[0].numpy()
    f = 440 * 2 ** ((63 - 69) / 12)
    n = np.arange(N)
    exp = 0.8 * np.sin(2 * np.pi * ((f / SR * n) % 1) + 0.5)
    assert np.abs(y - exp).max() < 1e-7


def test_whole_voice_silent_without_amp_routing(nebula_table):
    u = philox.sample_params(0, np.arange(4))
    for p in range(48, 68):
        if (p - 48) // 4 in (1, 3, 4):
            u[:, p] = 0.0
    y = voice.render_uniform(torch.tensor(u), np.arange(4), 4410, nebula_table)
    assert (y == 0).all()


def test_whole_voice_mixer_superposition(nebula_table):
    u = philox.sample_params(0, np.arange(6))
    ids = np.arange(6)
    full = voice.render_uniform(torch.tensor(u), ids, 20000, nebula_table, noise_seed=3)
    parts = 0
    for keep in (75, 76, 77):
        uu = u.copy()
        for p in (75, 76, 77):
            if p != keep:
                uu[:, p] = 0.0
        parts = parts + voice.render_uniform(torch.tensor(uu), ids, 20000, nebula_table, noise_seed=3)
    assert torch.allclose(full, parts, atol=1e-13)


def test_whole_voice_silent_tail(nebula_table):
    u = philox.sample_params(0, np.arange(32))
    y = voice.render_uniform(torch.tensor(u), np.arange(32), 176400, nebula_table)
    js = voice.silence_start(u, nebula_table)
    for b in range(32):
        start = int(math.ceil(js[b])) + 1
        if start * 100 < 176400:
            assert (y[b, start * 100:] == 0).all()
        # not silent before the note-off
        assert y[b, : max(1, int(js[b] * 100) - 5000)].abs().max() > 0 or js[b] < 60


def test_whole_voice_matches_scalar_brute_force():
    tab = W.curved_test_nebula().table()   # exercises curves and symmetric maps too
    u = philox.sample_params(11, np.arange(5))
    N = 1700
    y = voice.render_uniform(torch.tensor(u), np.arange(5), N, tab, sr=4410.0, rc=44.1, noise_seed=9)
    for b in range(5):
        ref = brute.render_one(u[b], b, N, tab, 4410.0, 44.1, 9)
        assert np.abs(y[b].numpy() - np.array(ref)).max() < 1e-11


def test_mode1_peak_normalisation(nebula_table):
    u = philox.sample_params(0, np.arange(16))
    u[:, 75:78] = 1 - 2**-24
    y0 = voice.render_uniform(torch.tensor(u), np.arange(16), 44100, nebula_table, mix_mode=0)
    y1 = voice.render_uniform(torch.tensor(u), np.arange(16), 44100, nebula_table, mix_mode=1)
    assert y1.abs().max() <= 1.0 + 1e-15
    pk = y0.abs().amax(-1)
    for b in range(16):
        if pk[b] <= 1:
            assert torch.equal(y0[b], y1[b])
        else:
            assert torch.allclose(y1[b], y0[b] / pk[b], atol=1e-15)
    assert (pk > 1).any()


def test_ragged_render_packs_uniform_renders(nebula_table):
    u = philox.sample_params(0, np.arange(6))
    L = np.array([4410, 8820, 4410, 17640, 8820, 4410])
    packed = voice.render(torch.tensor(u), np.arange(6), L, nebula_table)
    off = np.concatenate([[0], np.cumsum(L)])
    for b in range(6):
        one = voice.render_uniform(torch.tensor(u[b:b + 1]), [b], int(L[b]), nebula_table)[0]
        assert torch.equal(packed[off[b]:off[b + 1]], one)


def test_truncated_render_is_prefix_except_last_segment(nebula_table):
    u = philox.sample_params(0, np.arange(3))
    a = voice.render_uniform(torch.tensor(u), np.arange(3), 44100, nebula_table)
    b = voice.render_uniform(torch.tensor(u), np.arange(3), 88200, nebula_table)
    assert torch.allclose(a[:, :44000], b[:, :44000], atol=1e-12)


def test_train_test_split_rule():
    assert not voice.is_test(0) and not voice.is_test(9 * 1024 - 1)
    assert voice.is_test(9 * 1024) and voice.is_test(10 * 1024 - 1)
    assert not voice.is_test(10 * 1024)
    frac = np.mean([voice.is_test(g) for g in range(0, 102400, 7)])
    assert abs(frac - 0.1) < 0.01
