"""Pins of the resonant low-pass oracle (oracle/filter.py): the cookbook
section's frequency response (unit DC gain, a zero at Nyquist, gain Q at the
cutoff), scipy's lfilter for constant coefficients, a scalar brute force for
switched coefficients, the cutoff mapping and clamp, linearity in x, and the
autograd gradient against central differences."""
import math

import numpy as np
import scipy.signal
import torch

from oracle import filter as F

SR = 44100.0


def _H(b, a, w):
    z = np.exp(-1j * w)
    return (b[0] + b[1] * z + b[2] * z * z) / (1.0 + a[0] * z + a[1] * z * z)


def test_frequency_response_of_the_section():
    for f, q in ((100.0, 0.7), (1000.0, 4.0), (8000.0, 12.0), (15000.0, 0.5)):
        b0, b1, b2, a1, a2 = (c.item() for c in F.coefficients(torch.tensor([[f]], dtype=torch.float64), torch.tensor([q], dtype=torch.float64), SR))
        w0 = 2 * math.pi * f / SR
        assert abs(_H((b0, b1, b2), (a1, a2), 0.0) - 1.0) < 1e-12          # DC
        assert abs(_H((b0, b1, b2), (a1, a2), math.pi)) < 1e-12            # Nyquist
        assert abs(abs(_H((b0, b1, b2), (a1, a2), w0)) - q) < 1e-9 * q     # resonance at the cutoff
        # the poles lie inside the unit circle
        assert np.all(np.abs(np.roots([1.0, a1, a2])) < 1.0)


def test_constant_coefficients_match_lfilter():
    rng = np.random.default_rng(0)
    x = rng.standard_normal((3, 1000))
    cutoff, depth, q = np.array([60.0, 90.0, 110.0]), np.zeros(3), np.array([0.8, 3.0, 9.0])
    env = rng.uniform(size=(3, 10))
    y = F.lowpass(x, env, cutoff, depth, q, 100, SR).numpy()
    f = F.cutoff_hz(cutoff, depth, env, SR).numpy()
    for b in range(3):
        b0, b1, b2, a1, a2 = (c.numpy()[b, 0] for c in F.coefficients(torch.tensor(f), torch.tensor(q), SR))
        ref = scipy.signal.lfilter([b0, b1, b2], [1.0, a1, a2], x[b])
        assert np.max(np.abs(y[b] - ref)) < 1e-12 * max(1.0, np.max(np.abs(ref)))


def test_switched_coefficients_brute_force():
    rng = np.random.default_rng(1)
    N, period = 37, 8
    x = rng.standard_normal(N)
    env = rng.uniform(size=(1, 5))
    cutoff, depth, q = 70.0, 24.0, 2.5
    y = F.lowpass(x[None], env, [cutoff], [depth], [q], period, SR).numpy()[0]
    # scalar re-derivation with the period's coefficients taken afresh
    out, x1, x2, y1, y2 = [], 0.0, 0.0, 0.0, 0.0
    for n in range(N):
        m = cutoff + depth * env[0, n // period]
        f = min(max(440.0 * 2.0 ** ((m - 69.0) / 12.0), 10.0), 0.45 * SR)
        w = 2 * math.pi * f / SR
        al = math.sin(w) / (2 * q)
        a0 = 1 + al
        yn = ((1 - math.cos(w)) / 2 * x[n] + (1 - math.cos(w)) * x1 + (1 - math.cos(w)) / 2 * x2
              + 2 * math.cos(w) * y1 - (1 - al) * y2) / a0
        out.append(yn)
        x2, x1, y2, y1 = x1, x[n], y1, yn
    assert np.max(np.abs(y - np.array(out))) < 1e-13


def test_cutoff_mapping_and_clamp():
    f = F.cutoff_hz([69.0, 57.0, 69.0, 200.0, -100.0], [0.0, 12.0, -24.0, 0.0, 0.0],
                    np.array([[0.3], [1.0], [0.5], [0.0], [0.0]]), SR).numpy()[:, 0]
    assert abs(f[0] - 440.0) < 1e-12
    assert abs(f[1] - 440.0) < 1e-12                  # 57 + 12 * 1 = 69
    assert abs(f[2] - 220.0) < 1e-12                  # 69 - 24 * 0.5 = 57
    assert f[3] == 0.45 * SR and f[4] == 10.0


def test_linear_in_x_and_unit_step():
    rng = np.random.default_rng(2)
    x1, x2 = rng.standard_normal((2, 1, 500))
    env = rng.uniform(size=(1, 5))
    args = (env, [80.0], [12.0], [1.5], 100, SR)
    y = F.lowpass(2.0 * x1 - 3.0 * x2, *args).numpy()
    assert np.allclose(y, 2.0 * F.lowpass(x1, *args).numpy() - 3.0 * F.lowpass(x2, *args).numpy(),
                       atol=1e-12)
    step = F.lowpass(np.ones((1, 20000)), np.zeros((1, 200)), [90.0], [0.0], [0.7071], 100, SR).numpy()
    assert abs(step[0, -1] - 1.0) < 1e-9              # unit DC gain


def test_autograd_matches_central_differences():
    rng = np.random.default_rng(3)
    B, N, period = 2, 300, 50
    x = torch.tensor(rng.standard_normal((B, N)), requires_grad=True)
    env = torch.tensor(rng.uniform(size=(B, 6)), requires_grad=True)
    p = torch.tensor([[62.0, 18.0, 2.0], [75.0, -10.0, 6.0]], dtype=torch.float64, requires_grad=True)
    w = torch.tensor(rng.standard_normal((B, N)))

    def loss(x, env, p):
        return (w * F.lowpass(x, env, p[:, 0], p[:, 1], p[:, 2], period, SR)).sum()

    gx, genv, gp = torch.autograd.grad(loss(x, env, p), (x, env, p))
    h = 1e-5
    args = {"x": x.detach(), "env": env.detach(), "p": p.detach()}
    for key, g, idx in (("p", gp, [(0, 0), (0, 1), (0, 2), (1, 0), (1, 1), (1, 2)]),
                        ("env", genv, [(0, 0), (1, 3), (0, 5)]), ("x", gx, [(0, 0), (1, 123), (1, 299)])):
        for i in idx:
            d = torch.zeros_like(args[key])
            d[i] = h
            up, dn = dict(args), dict(args)
            up[key], dn[key] = args[key] + d, args[key] - d
            with torch.no_grad():
                fd = (loss(**up) - loss(**dn)) / (2 * h)
            assert abs(fd.item() - g[i].item()) < 1e-6 * max(1.0, abs(fd.item())), (key, i, fd, g[i])
