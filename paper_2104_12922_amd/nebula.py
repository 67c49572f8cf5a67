"""Sets of sounds compared by maximum mean discrepancy, and the nebula search
that tunes the sampling curves against it (Sections 5 and 6).

The MMD of two sets X (n sounds) and Y (m sounds) over the L1 distance
between embeddings is

    MMD(X, Y) = 2 S(X, Y) / (n m) - S(X, X) / n^2 - S(Y, Y) / m^2,
    S(A, B)   = sum over all pairs (a, b) of ||a - b||_1,

the paper's equation "mmd" (written there for n = m), an energy distance that
is 0 for identical sets.  A sound's embedding is its 128 x 64 log-mel
spectrogram.  The pair sums run in libsynth.so (`synth_mmd_l1`).

A nebula assigns each of the Voice's 78 parameters a range, a curve and a
symmetry flag (Section 3.3).  `NebulaSearch` tunes the curves of chosen
parameters, sampled log-uniformly in [0.1, 10], to minimise (or maximise) the
MMD between a set of sounds drawn from the nebula and a target set: random
trials, then CMA-ES trials, then the best candidates re-scored over fresh
draws, as Section 6 describes.  Each trial draws, renders, embeds and scores
its sounds on the device; only the curve vectors and the scalar MMD cross to
the host.
"""
from __future__ import annotations

import ctypes
import math
from dataclasses import dataclass, field

import numpy as np
import torch

from . import _dev_ptr, _native, _stream

F32 = torch.float32
F64 = torch.float64
CURVE_LO, CURVE_HI = 0.1, 10.0
MAX_SET = 1 << 17          # sounds per set (synth_mmd_l1)


def _sig(L):
    vp, i64, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_size_t
    L.synth_l1_pair_sum_workspace.restype = sz
    L.synth_l1_pair_sum_workspace.argtypes = [i64, i64, i64]
    L.synth_mmd_l1_workspace.restype = sz
    L.synth_mmd_l1_workspace.argtypes = [i64, i64, i64]
    L.synth_l1_pair_sum.restype = ctypes.c_int
    L.synth_l1_pair_sum.argtypes = [vp, i64, i64, vp, i64, i64, i64, vp, sz, vp, vp]
    L.synth_mmd_l1.restype = ctypes.c_int
    L.synth_mmd_l1.argtypes = [vp, i64, vp, i64, i64, vp, sz, vp, vp]
    return L


_L = None


def lib():
    global _L
    if _L is None:
        _L = _sig(_native.lib())
    return _L


def _rows(t, name):
    if t.dim() != 2 or t.dtype != F32 or not t.is_cuda:
        raise ValueError(f"{name} must be a float32 [rows, dim] device tensor")
    if t.stride(1) != 1:
        raise ValueError(f"{name} must have unit column stride")
    return t


class _Workspace:
    def __init__(self):
        self.buf = None

    def get(self, need, device):
        if need and (self.buf is None or self.buf.numel() < need or self.buf.device != device):
            self.buf = torch.empty(need, dtype=torch.uint8, device=device)
        return (self.buf.data_ptr(), self.buf.numel()) if need else (None, 0)


_WS = _Workspace()


def l1_pair_sum(A: torch.Tensor, B: torch.Tensor, out: torch.Tensor | None = None,
                workspace: _Workspace | None = None) -> torch.Tensor:
    """S(A, B) = sum over all row pairs of the L1 distance (0-d float64)."""
    A, B = _rows(A, "A"), _rows(B, "B")
    if A.shape[1] != B.shape[1]:
        raise ValueError("A and B must have the same number of columns")
    n, m, dim = A.shape[0], B.shape[0], A.shape[1]
    if out is None:
        out = torch.empty((), dtype=F64, device=A.device)
    ws = (workspace or _WS).get(lib().synth_l1_pair_sum_workspace(n, m, dim), A.device)
    _native.check("synth_l1_pair_sum", lib().synth_l1_pair_sum(
        A.data_ptr() if A.numel() else None, max(A.stride(0), dim), n,
        B.data_ptr() if B.numel() else None, max(B.stride(0), dim), m, dim, *ws,
        _dev_ptr(out, "out", F64, 1), _stream(A.device)))
    return out


def mmd_l1(X: torch.Tensor, Y: torch.Tensor, out: torch.Tensor | None = None,
           workspace: _Workspace | None = None) -> torch.Tensor:
    """float64 [4] device tensor (MMD(X, Y), S(X, Y), S(X, X), S(Y, Y))."""
    X, Y = _rows(X, "X").contiguous(), _rows(Y, "Y").contiguous()
    if X.shape[1] != Y.shape[1]:
        raise ValueError("X and Y must have the same number of columns")
    n, m, dim = X.shape[0], Y.shape[0], X.shape[1]
    if not (1 <= n <= MAX_SET and 1 <= m <= MAX_SET):
        raise ValueError(f"MMD needs two non-empty sets of at most {MAX_SET} sounds")
    if out is None:
        out = torch.empty(4, dtype=F64, device=X.device)
    ws = (workspace or _WS).get(lib().synth_mmd_l1_workspace(n, m, dim), X.device)
    _native.check("synth_mmd_l1", lib().synth_mmd_l1(
        X.data_ptr(), n, Y.data_ptr(), m, dim, *ws, _dev_ptr(out, "out", F64, 4),
        _stream(X.device)))
    return out


def with_curves(nebula_table, params, log10_curves) -> np.ndarray:
    """Copy of a [78, 4] nebula table with the curves of `params` set to
    10 ** log10_curves."""
    tab = np.array(nebula_table, dtype=np.float64).reshape(-1, 4).copy()
    tab[np.asarray(params, dtype=np.int64), 2] = 10.0 ** np.asarray(log10_curves, dtype=np.float64)
    return tab


class SoundSets:
    """Draws, renders and embeds sets of sounds from a nebula on the device:
    set k of a seed is the voices g = k * stride + [0, n) of the corpus keyed
    by that seed (parameters from the counter-based generator, n_samples
    each), embedded as log-mel spectrograms [n, 8192]."""

    def __init__(self, n_sounds: int = 256, n_samples: int = 176400, seed: int = 30,
                 sample_rate: float = 44100.0, device="cuda", stride: int = 1 << 20):
        from .learned import LogMel
        if n_sounds > stride:
            raise ValueError("n_sounds must not exceed the stride between sets")
        self.n, self.samples, self.seed, self.sr = int(n_sounds), int(n_samples), int(seed), float(sample_rate)
        self.device = torch.device(device)
        self.stride = int(stride)
        self.logmel = LogMel(sample_rate, device=self.device)
        self._u = torch.empty(self.n, 78, dtype=F32, device=self.device)
        self._audio = torch.empty(self.n, self.samples, dtype=F32, device=self.device)

    def embed(self, nebula_table, k: int, out: torch.Tensor | None = None) -> torch.Tensor:
        from . import synth_render, synth_sample_params
        g0 = int(k) * self.stride
        synth_sample_params(self.seed, first_g=g0, batch=self.n, out=self._u)
        synth_render(self._u, nebula_table, n_samples=self.samples, first_g=g0,
                     noise_seed=self.seed, sample_rate=self.sr, out=self._audio.view(-1))
        return self.logmel(self._audio, out=out)


@dataclass
class Trial:
    number: int
    phase: str                  # "random" or "cmaes"
    log10_curves: np.ndarray
    value: float


@dataclass
class SearchResult:
    best_log10_curves: np.ndarray
    best_mean: float            # mean MMD over the re-scoring draws
    rescored: list = field(default_factory=list)   # (trial number, mean, std) of the top candidates
    trials: list = field(default_factory=list)


class NebulaSearch:
    """Tune the curves of `params` (indices into the Voice's 78 parameters) of
    `base_table` against a target set of embeddings [m, 8192] (device float32).

    Trial t scores the sound set drawn with set index t (fresh sounds every
    trial) against `target_per_trial` target rows picked by a seeded
    permutation (all rows if fewer).  direction "minimize" makes the nebula
    sound like the target; "maximize" pushes it away."""

    def __init__(self, base_table, target: torch.Tensor, params=None, sets: SoundSets | None = None,
                 target_per_trial: int = 256, direction: str = "minimize", seed: int = 0):
        if direction not in ("minimize", "maximize"):
            raise ValueError("direction must be 'minimize' or 'maximize'")
        self.base = np.array(base_table, dtype=np.float64).reshape(-1, 4)
        self.params = np.arange(self.base.shape[0]) if params is None else np.asarray(params, dtype=np.int64)
        self.target = _rows(target, "target").contiguous()
        self.sets = sets or SoundSets(device=target.device)
        self.m = min(int(target_per_trial), self.target.shape[0])
        self.sign = 1.0 if direction == "minimize" else -1.0
        self.seed = int(seed)
        self.rng = np.random.default_rng(seed)
        self._x = torch.empty(self.sets.n, self.target.shape[1], dtype=F32, device=self.target.device)
        self._out = torch.empty(4, dtype=F64, device=self.target.device)
        self._ws = _Workspace()
        self.trials: list[Trial] = []

    def score(self, log10_curves, k: int) -> float:
        """MMD between set k of the candidate nebula and the target rows of draw k."""
        tab = with_curves(self.base, self.params, log10_curves)
        X = self.sets.embed(tab, k, out=self._x)
        if self.m < self.target.shape[0]:
            g = torch.Generator().manual_seed(self.seed * 1000003 + int(k))
            rows = torch.randperm(self.target.shape[0], generator=g)[:self.m].to(self.target.device)
            Y = self.target.index_select(0, rows)
        else:
            Y = self.target
        return float(mmd_l1(X, Y, out=self._out, workspace=self._ws)[0].item())

    def _run_trial(self, phase, z):
        k = len(self.trials)
        v = self.score(z, k)
        self.trials.append(Trial(k, phase, np.array(z), v))
        return v

    def run(self, n_random: int = 200, n_cmaes: int = 800, top_k: int = 25, rescore: int = 30,
            sigma0: float | None = None, callback=None) -> SearchResult:
        """Random trials (log10 curves uniform in [-1, 1]), CMA-ES trials from
        the best random trial, then the top_k trials re-scored on the same
        `rescore` fresh draws; the lowest mean (highest, maximising) wins."""
        from .cmaes import CMAES
        lo, hi = math.log10(CURVE_LO), math.log10(CURVE_HI)
        d = self.params.size
        for _ in range(n_random):
            v = self._run_trial("random", self.rng.uniform(lo, hi, d))
            if callback:
                callback(self.trials[-1])
        if n_cmaes > 0:
            start = (min(self.trials, key=lambda t: self.sign * t.value).log10_curves
                     if self.trials else np.zeros(d))
            es = CMAES(start, sigma0 if sigma0 is not None else (hi - lo) / 6.0, lo, hi,
                       seed=self.seed + 1)
            done = 0
            while done < n_cmaes:
                cand = es.ask()
                vals = []
                for z in cand:
                    if done < n_cmaes:
                        vals.append(self.sign * self._run_trial("cmaes", z))
                        if callback:
                            callback(self.trials[-1])
                    else:                       # budget spent mid-generation: rank last
                        vals.append(math.inf)
                    done += 1
                es.tell(vals)
        ranked = sorted(self.trials, key=lambda t: self.sign * t.value)[:max(1, top_k)]
        # every candidate is re-scored on the same fresh draws (common random numbers)
        base_k = len(self.trials)
        rescored = []
        for t in ranked:
            vals = [self.score(t.log10_curves, base_k + r) for r in range(rescore)]
            rescored.append((t.number, float(np.mean(vals)), float(np.std(vals))))
        best = min(rescored, key=lambda r: self.sign * r[1])
        return SearchResult(self.trials[best[0]].log10_curves.copy(), best[1], rescored,
                            list(self.trials))
