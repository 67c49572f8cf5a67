"""Maximum mean discrepancy between two sets of sounds (float64, numpy).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

Section 5 of the paper compares sets of sounds with the maximum mean
discrepancy over an auditory distance d between embeddings (its equation
"mmd", for |X| = |Y| = n):

    MMD(X, Y) = 1/(n n) sum_{i,j} [ 2 d(x_i, y_j) - d(x_i, x_j) - d(y_i, y_j) ]

with d the L1 distance between embeddings (Section 4 prefers L1 to L2).
Readings taken here: the paper's embedding (OpenL3) is not available, so the
embedding of a sound is its 128 x 64 log-mel feature vector (the features the
learned proposal reads); for sets of different sizes n, m each double sum is
normalised by its own number of pairs,

    MMD(X, Y) = 2/(n m) sum d(x_i, y_j) - 1/n^2 sum d(x_i, x_j) - 1/m^2 sum d(y_i, y_j),

which is the paper's expression when n = m.  The sums include i = j (where
d = 0), as the printed formula does.  For the L1 distance this is the energy
distance between the two empirical distributions, which is never negative.
"""
from __future__ import annotations

import numpy as np


def l1_distance_sum(A, B) -> float:
    """sum_{i,j} ||A_i - B_j||_1 over all pairs of rows (float64)."""
    A = np.asarray(A, dtype=np.float64)
    B = np.asarray(B, dtype=np.float64)
    total = 0.0
    for a in A:                         # one row against all rows: [m, dim]
        total += float(np.abs(B - a[None, :]).sum())
    return total


def mmd(X, Y) -> float:
    """MMD(X, Y) with the L1 distance; X [n, dim], Y [m, dim]."""
    n, m = len(X), len(Y)
    return (2.0 * l1_distance_sum(X, Y) / (n * m) - l1_distance_sum(X, X) / (n * n)
            - l1_distance_sum(Y, Y) / (m * m))
