"""Launch-plan autotuner for the batched render.

A plan is (runs_per_segment, slices_per_voice, persistent, grid_blocks,
carries) of `synth_render_plan` (carries: split voices start from
precomputed chunk carries instead of walking the earlier chunks; a 4-tuple
means carries off).  Plans with the same runs per segment render identical
bits; changing the runs per segment regroups the float64 phase sums, which
moves samples by float32 rounding only (every plan is held to the same parity
tolerance against the oracle), so the choice is one of speed.  The tuner times each candidate plan on the caller's
own batch (HIP events on the current stream, median of `reps` launches after
one warm-up, the smaller of two rounds), keeps the fastest per batch shape, and can save and reload its
table as JSON.  Tuning happens outside any timed region; a tuned render is
one `synth_render_plan` call.
"""
from __future__ import annotations

import json
import os

import numpy as np
import torch

from . import synth_render_plan


def default_candidates(batch: int, uniform: bool, nchunks: int | None = None):
    """Plans worth timing (the library's default plan first): 4 or 2 runs per
    control period; one workgroup per voice, or a persistent grid of 4-16
    workgroups per CU (256 CUs); batches of up to 16384 voices also try
    splitting each voice over several workgroups (slices: 2-32 for small
    uniform batches, at most the voice's chunk count; 2-4 otherwise), which
    evens out the load when lengths differ.  Split plans render with the
    chunk-start carries computed first."""
    c = []
    for rps in (4, 2):
        c.append((rps, 1, 0, 0))
        for g in (1024, 2048, 4096):
            if g < batch:
                c.append((rps, 1, 1, g))
        if batch < 256 and uniform:
            for sl in (2, 4, 8, 16, 32):
                if nchunks is None or sl <= nchunks:
                    c.append((rps, sl, 0, 0, 1))
        elif batch <= 16384:
            for sl in (2, 3, 4):
                c.append((rps, sl, 0, 0, 0))
                c.append((rps, sl, 0, 0, 1))
    return c


def _plan5(plan):
    return tuple(plan) + (0,) * (5 - len(plan))


class RenderTuner:
    def __init__(self, reps: int = 5, candidates=None, margin: float = 0.02):
        self.reps = reps
        self.margin = margin
        self.candidates = candidates
        self.table: dict[str, tuple] = {}
        self.timings: dict[str, dict] = {}

    @staticmethod
    def key(batch: int, n_samples: int | None, offsets: torch.Tensor | None) -> str:
        """Batch shape: uniform length, or the histogram of ragged lengths (the
        plan's speed depends on the mix of lengths, not on their order)."""
        if offsets is None:
            return f"u:{batch}:{int(n_samples)}"
        lens = torch.diff(offsets).cpu().numpy().astype(np.int64)
        vals, counts = np.unique(lens, return_counts=True)
        h = hash((tuple(vals.tolist()), tuple(counts.tolist()))) & 0xFFFFFFFF
        return f"r:{batch}:{int(lens.sum())}:{h:08x}"

    def tune(self, params, nebula, n_samples=None, offsets=None, out=None, key=None, **kw):
        B = params.shape[0]
        k = key if key is not None else self.key(B, n_samples, offsets)
        nch = None
        if offsets is None and n_samples:
            q = int(round(kw.get("sample_rate", 44100.0) / kw.get("control_rate", 441.0)))
            periods = -(-int(n_samples) // q)
            nch = -(-periods // 62)                      # chunks of 62 control periods
        cands = self.candidates or default_candidates(B, offsets is None, nch)
        stream = torch.cuda.current_stream()
        times = {}
        # Two rounds over all candidates, each plan's median per round, the
        # smaller kept: a plan timed first would otherwise carry the GPU's
        # ramp from idle to full clock.
        for _ in range(2):
            for plan in cands:
                rps, sl, pers, grid, car = _plan5(plan)

                def run():
                    return synth_render_plan(params, nebula, rps, sl, persistent=bool(pers),
                                             grid_blocks=grid, n_samples=n_samples, offsets=offsets,
                                             out=out, carries=bool(car), **kw)
                out = run()                          # warm-up (and the output buffer)
                ts = []
                for _ in range(self.reps):
                    a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
                    a.record(stream)
                    run()
                    b.record(stream)
                    b.synchronize()
                    ts.append(a.elapsed_time(b))
                times[plan] = min(times.get(plan, float("inf")), float(np.median(ts)))
        best = min(times, key=times.get)
        default = cands[0]
        if default in times and times[best] > (1.0 - self.margin) * times[default]:
            best = default                     # keep the default plan unless clearly faster
        self.table[k] = best
        self.timings[k] = {",".join(map(str, p)): t for p, t in times.items()}
        return best, times

    def plan_for(self, params, nebula, n_samples=None, offsets=None, key=None, **kw):
        """The plan for this batch shape, tuning it on first sight.  `key` lets a
        caller that knows its shape name it (avoids reading the offsets back)."""
        k = key if key is not None else self.key(params.shape[0], n_samples, offsets)
        if k not in self.table:
            self.tune(params, nebula, n_samples=n_samples, offsets=offsets, key=k, **kw)
        return self.table[k]

    def render(self, params, nebula, n_samples=None, offsets=None, out=None, key=None, **kw):
        rps, sl, pers, grid, car = _plan5(self.plan_for(params, nebula, n_samples=n_samples,
                                                         offsets=offsets, key=key, **kw))
        return synth_render_plan(params, nebula, rps, sl, persistent=bool(pers), grid_blocks=grid,
                                 n_samples=n_samples, offsets=offsets, out=out,
                                 carries=bool(car), **kw)

    def save(self, path: str):
        with open(path, "w") as f:
            json.dump({"table": {k: list(v) for k, v in self.table.items()},
                       "timings_ms": self.timings}, f, indent=1)

    def load(self, path: str):
        if os.path.exists(path):
            with open(path) as f:
                d = json.load(f)
            self.table.update({k: tuple(v) for k, v in d.get("table", {}).items()})
