"""Pins of the oracle's counter-based generator (parameter draw and noise)."""
import os

import numpy as np
import pytest
from scipy import stats

from oracle import philox

GOLDEN = os.path.join(os.path.dirname(__file__), "golden", "philox4x32_10_kat.txt")


def _kat():
    rows = []
    for line in open(GOLDEN):
        line = line.strip()
        if not line or line.startswith("#"):
            continue
        w = [int(x, 16) for x in line.split()]
        rows.append((w[0:4], w[4:6], w[6:10]))
    return rows


@pytest.mark.parametrize("ctr,key,out", _kat())
def test_philox_known_answers(ctr, key, out):
    got = philox.philox4x32(np.array(ctr, np.uint64), np.array(key, np.uint64))
    assert [int(x) for x in got] == out


def test_philox_vectorised_matches_rowwise():
    rng = np.random.default_rng(0)
    ctr = rng.integers(0, 2**32, size=(37, 4), dtype=np.uint64)
    key = rng.integers(0, 2**32, size=(2,), dtype=np.uint64)
    allv = philox.philox4x32(ctr, key)
    for i in range(37):
        assert (philox.philox4x32(ctr[i], key) == allv[i]).all()


def test_u24_exact_in_float32_and_range():
    u = philox.sample_params(7, np.arange(64))
    assert u.shape == (64, 78)
    assert (u >= 0).all() and (u <= 1 - 2**-24).all()
    assert (u.astype(np.float32).astype(np.float64) == u).all()
    assert (u * 2**24 == np.floor(u * 2**24)).all()
    assert philox.u24(0xFFFFFFFF) == 1 - 2**-24 and philox.u24(0xFF) == 0.0


def test_param_draw_counter_layout():
    # word p & 3 of counter (g lo, g hi, p >> 2, 0), key = seed
    seed, g = 0x1234_5678_9ABC, (1 << 33) + 5
    u = philox.sample_params(seed, [g])[0]
    for p in (0, 3, 4, 41, 77):
        w = philox.philox4x32(np.array([g & 0xFFFFFFFF, g >> 32, p >> 2, 0], np.uint64),
                              np.array([seed & 0xFFFFFFFF, seed >> 32], np.uint64))[p & 3]
        assert u[p] == (int(w) >> 8) / 2**24


def test_param_draw_independent_of_batching():
    full = philox.sample_params(3, np.arange(100))
    part = philox.sample_params(3, np.arange(40, 57))
    assert (full[40:57] == part).all()
    assert not (philox.sample_params(4, np.arange(10)) == full[:10]).all()


def test_param_draw_is_uniform():
    u = philox.sample_params(0, np.arange(4000)).reshape(-1)
    assert abs(u.mean() - 0.5) < 3e-3
    assert abs(u.var() - 1 / 12) < 2e-3
    assert stats.kstest(u, "uniform").pvalue > 1e-3


def test_noise_statistics_and_layout():
    x = philox.noise(0, 5, 200_000)
    assert abs(x.mean()) < 5e-3
    assert abs(x.var() - 1 / 3) < 5e-3
    assert (x > -1).all() and (x < 1).all()
    # 8 samples per generator call: low half of word 0 first
    w = philox.philox4x32(np.array([5, 0, 1, 1], np.uint64), np.array([0, 0], np.uint64))
    h = philox.noise_halfwords(0, 5, 16)[8:16]
    exp = [int(w[k // 2]) >> (16 * (k & 1)) & 0xFFFF for k in range(8)]
    assert list(h) == exp
    # distinct voices are decorrelated
    y = philox.noise(0, 6, 200_000)
    assert abs(np.corrcoef(x, y)[0, 1]) < 0.01
    # noise stream (counter word 3 = 1) differs from the parameter stream
    assert not np.array_equal(philox.noise_halfwords(0, 0, 8), philox.noise_halfwords(1, 0, 8))
