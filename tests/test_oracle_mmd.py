"""Pins of the MMD oracle (Section 5, equation "mmd", L1 distance): closed
forms on tiny sets, a pure-Python brute force, identity and symmetry, scale
covariance, and non-negativity (the L1 energy distance)."""
import itertools

import numpy as np

from oracle import mmd as M


def brute(X, Y):
    d = lambda a, b: sum(abs(p - q) for p, q in zip(a, b))
    n, m = len(X), len(Y)
    sxy = sum(d(a, b) for a, b in itertools.product(X, Y))
    sxx = sum(d(a, b) for a, b in itertools.product(X, X))
    syy = sum(d(a, b) for a, b in itertools.product(Y, Y))
    return 2 * sxy / (n * m) - sxx / (n * n) - syy / (m * m)


def test_closed_forms():
    assert M.mmd([[0.0]], [[3.0]]) == 6.0                       # 2 |a - b|, singletons
    # X = {0, 2}, Y = {1}: 2 (1 + 1)/2 - (0 + 2 + 2 + 0)/4 - 0 = 1
    assert M.mmd([[0.0], [2.0]], [[1.0]]) == 1.0
    # two dimensions add: d is L1
    assert M.mmd([[0.0, 0.0]], [[1.0, -2.0]]) == 6.0
    # the paper's form for n = m: 1/(n n) sum (2 d(x, y) - d(x, x') - d(y, y'))
    X = np.array([[0.0, 1.0], [2.0, 0.0]])
    Y = np.array([[1.0, 1.0], [0.0, 3.0]])
    n = 2
    paper = sum(2 * np.abs(X[i] - Y[j]).sum() - np.abs(X[i] - X[j]).sum() - np.abs(Y[i] - Y[j]).sum()
                for i in range(n) for j in range(n)) / (n * n)
    assert abs(M.mmd(X, Y) - paper) < 1e-15


def test_brute_force_identity_symmetry_scale_and_sign():
    rng = np.random.default_rng(0)
    for n, m, dim in ((3, 5, 4), (7, 2, 9), (4, 4, 1)):
        X = rng.standard_normal((n, dim))
        Y = rng.standard_normal((m, dim)) + 0.3
        v = M.mmd(X, Y)
        assert abs(v - brute(X.tolist(), Y.tolist())) < 1e-12 * max(1.0, abs(v))
        assert abs(v - M.mmd(Y, X)) < 1e-12
        assert abs(M.mmd(2.5 * X, 2.5 * Y) - 2.5 * v) < 1e-12 * max(1.0, v)
        assert M.mmd(X, X) == 0.0
        assert v > 0.0
