"""CMA-ES over a box, the sampler of the nebula search (Section 6: random
trials, then covariance-matrix-adaptation trials, over curve hyperparameters).

Host-side search logic only (a few hundred floats per generation); the
objective it drives renders and scores sounds on the device.  The update is
the (mu/mu_w, lambda)-CMA-ES with cumulative step-size adaptation and
rank-one plus rank-mu covariance updates, with the default strategy
parameters of N. Hansen, "The CMA Evolution Strategy: A Tutorial"
(arXiv:1604.00772, 2016), Table 1 (positive recombination weights only).

Box constraints: the strategy runs unconstrained in y, and a candidate is
evaluated at the reflection of y into the box (the triangle wave that folds
the real line onto [lo, hi], identity inside the box), so every evaluated
point is feasible, the objective seen by the strategy is continuous, and no
clipping or penalty distorts the step-size and covariance updates.
"""
from __future__ import annotations

import math

import numpy as np


class CMAES:
    """Minimiser for objectives over [lo, hi]^n.  Use ask() for a generation's
    candidates (points inside the box to evaluate), then tell(values) with
    their objective values in the same order."""

    def __init__(self, mean, sigma: float, lo, hi, seed: int = 0, popsize: int | None = None):
        self.m = np.array(mean, dtype=np.float64)
        n = self.n = self.m.size
        self.lo = np.broadcast_to(np.asarray(lo, dtype=np.float64), (n,)).copy()
        self.hi = np.broadcast_to(np.asarray(hi, dtype=np.float64), (n,)).copy()
        if np.any(self.hi <= self.lo):
            raise ValueError("every upper bound must exceed its lower bound")
        self.m = np.clip(self.m, self.lo, self.hi)
        self.sigma = float(sigma)
        self.rng = np.random.default_rng(seed)
        lam = popsize or 4 + int(3 * math.log(n))
        mu = lam // 2
        w = math.log(mu + 0.5) - np.log(np.arange(1, mu + 1))
        self.w = w / w.sum()
        self.lam, self.mu = lam, mu
        self.mueff = 1.0 / float(np.sum(self.w ** 2))
        me = self.mueff
        self.cs = (me + 2.0) / (n + me + 5.0)
        self.ds = 1.0 + 2.0 * max(0.0, math.sqrt((me - 1.0) / (n + 1.0)) - 1.0) + self.cs
        self.cc = (4.0 + me / n) / (n + 4.0 + 2.0 * me / n)
        self.c1 = 2.0 / ((n + 1.3) ** 2 + me)
        self.cmu = min(1.0 - self.c1, 2.0 * (me - 2.0 + 1.0 / me) / ((n + 2.0) ** 2 + me))
        self.chin = math.sqrt(n) * (1.0 - 1.0 / (4.0 * n) + 1.0 / (21.0 * n * n))
        self.pc = np.zeros(n)
        self.ps = np.zeros(n)
        self.C = np.eye(n)
        self.B = np.eye(n)
        self.D = np.ones(n)
        self.gen = 0
        self._pending = None

    def _eigen(self):
        self.C = np.triu(self.C) + np.triu(self.C, 1).T     # keep it symmetric
        d2, self.B = np.linalg.eigh(self.C)
        self.D = np.sqrt(np.maximum(d2, 1e-300))

    def fold(self, x) -> np.ndarray:
        """Reflection of x into [lo, hi] (period 2 (hi - lo))."""
        w = self.hi - self.lo
        t = np.mod(np.asarray(x, dtype=np.float64) - self.lo, 2.0 * w)
        return self.lo + np.where(t <= w, t, 2.0 * w - t)

    @property
    def mean(self) -> np.ndarray:
        """The distribution mean, folded into the box."""
        return self.fold(self.m)

    def ask(self) -> np.ndarray:
        """lambda candidates [lambda, n] inside the box."""
        z = self.rng.standard_normal((self.lam, self.n))
        y = (z * self.D) @ self.B.T                          # y ~ N(0, C)
        self._pending = y
        return self.fold(self.m + self.sigma * y)

    def tell(self, values) -> None:
        if self._pending is None:
            raise RuntimeError("tell() without ask()")
        y = self._pending
        self._pending = None
        f = np.asarray(values, dtype=np.float64)
        if f.shape != (self.lam,):
            raise ValueError(f"expected {self.lam} values")
        order = np.argsort(f, kind="stable")
        ysel = y[order[:self.mu]]
        yw = self.w @ ysel
        n = self.n
        self.m = self.m + self.sigma * yw
        # C^(-1/2) yw = B D^(-1) B^T yw
        cinv_yw = self.B @ ((self.B.T @ yw) / self.D)
        self.ps = (1.0 - self.cs) * self.ps + math.sqrt(self.cs * (2.0 - self.cs) * self.mueff) * cinv_yw
        self.gen += 1
        ps_norm = float(np.linalg.norm(self.ps))
        hs = ps_norm / math.sqrt(1.0 - (1.0 - self.cs) ** (2 * self.gen)) < (1.4 + 2.0 / (n + 1.0)) * self.chin
        self.pc = (1.0 - self.cc) * self.pc + (hs * math.sqrt(self.cc * (2.0 - self.cc) * self.mueff)) * yw
        dh = (1.0 - hs) * self.cc * (2.0 - self.cc)
        rank_mu = (ysel.T * self.w) @ ysel
        self.C = ((1.0 + self.c1 * dh - self.c1 - self.cmu) * self.C
                  + self.c1 * np.outer(self.pc, self.pc) + self.cmu * rank_mu)
        self.sigma *= math.exp((self.cs / self.ds) * (ps_norm / self.chin - 1.0))
        self._eigen()
