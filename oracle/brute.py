"""Scalar pure-Python Voice render for tiny inputs (a second, loop-by-loop
statement of the same definitions as ``oracle.voice``; it pins the vectorised
oracle's indexing, shifts and broadcasting).  TEST INFRASTRUCTURE ONLY.

Everything is a per-sample Python loop with ``math`` functions, following the
signal order of the Voice (Section 3.2).  Only for N of a few thousand samples.
"""
from __future__ import annotations

import math

from .philox import noise as philox_noise


def _map(u, row):
    lo, hi, c, sym = row
    if sym > 0.5:
        d = 2.0 * u - 1.0
        w = abs(d) if c == 1.0 else abs(d) ** (1.0 / c)
        s = 1.0 if d > 0 else (-1.0 if d < 0 else 0.0)
        return lo + (hi - lo) * (1.0 + s * w) / 2.0
    w = u if c == 1.0 else u ** (1.0 / c)
    return lo + (hi - lo) * w


def _ramp(j, start, length):
    if length > 0:
        return min(1.0, max(0.0, (j - start) / length))
    return 1.0 if j >= start else 0.0


def _env(j, a, d, s, r, alpha, off, rc):
    A, D, R, O = a * rc, d * rc, r * rc, off * rc
    att = _ramp(j, 0.0, A)
    dec = _ramp(j, A, D)
    rel = _ramp(j, O, R)
    return (att ** alpha) * (s + (1.0 - s) * (1.0 - dec) ** alpha) * (1.0 - rel) ** alpha


def render_one(u, g, N, table, sr, rc, noise_seed):
    """One voice, N samples, as a Python list of floats."""
    q = int(round(sr / rc))
    v = [_map(float(u[p]), [float(x) for x in table[p]]) for p in range(78)]
    J = -(-N // q)
    off = v[1]
    envs = [[_env(j, *v[b:b + 5], off, rc) for j in range(J)] for b in (2, 7, 12, 17, 22, 27)]
    lfos = []
    for i, b in enumerate((32, 40)):
        rate, depth, ph0 = v[b], v[b + 1], v[b + 2]
        w = v[b + 3:b + 8]
        ws = sum(w)
        th = ph0 / (2 * math.pi)
        out = []
        for j in range(J):
            ph = th - math.floor(th)
            shapes = [(1 + math.sin(2 * math.pi * ph)) / 2, 1 - abs(2 * ph - 1), ph, 1 - ph,
                      1.0 if ph < 0.5 else 0.0]
            val = sum(wk * sk for wk, sk in zip(w, shapes)) / ws if ws > 0 else 0.0
            out.append(val * envs[3 + 2 * i][j])
            th += max(0.0, rate + depth * envs[2 + 2 * i][j]) / rc
        lfos.append(out)
    xs = [envs[0], envs[1], lfos[0], lfos[1]]
    ys = []
    for o in range(5):
        G = v[48 + 4 * o:52 + 4 * o]
        norm = max(1.0, sum(G))
        ys.append([sum(G[i] * xs[i][j] for i in range(4)) / norm for j in range(J)])

    def up(row, n):
        j0 = n // q
        t = (n - j0 * q) / q
        return (1 - t) * row[j0] + t * row[min(j0 + 1, J - 1)]

    def hz(m):
        return min(sr / 2, 440.0 * 2.0 ** ((m - 69.0) / 12.0))

    m_hi = max(0.0, v[0] + v[71] + max(0.0, v[72]))
    f_hi = hz(m_hi)
    K = 12000.0 / (f_hi * math.log10(f_hi))
    s = v[74]
    nz = philox_noise(noise_seed, g, N)
    th1 = v[70] / (2 * math.pi)
    th2 = v[73] / (2 * math.pi)
    y = []
    for n in range(N):
        p1 = th1 - math.floor(th1)
        p2 = th2 - math.floor(th2)
        x1 = math.sin(2 * math.pi * p1)
        x2 = (1 - s / 2) * math.tanh(K * math.sin(2 * math.pi * p2)) * (1 + s * math.cos(2 * math.pi * p2))
        x3 = float(nz[n])
        y.append(v[75] * x1 * up(ys[1], n) + v[76] * x2 * up(ys[3], n) + v[77] * x3 * up(ys[4], n))
        th1 += hz(v[0] + v[68] + v[69] * up(ys[0], n)) / sr
        th2 += hz(v[0] + v[71] + v[72] * up(ys[2], n)) / sr
    return y
