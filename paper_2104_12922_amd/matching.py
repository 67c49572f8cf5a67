"""Sound matching: estimate the synthesizer parameters of target sounds.

The paper motivates the corpus with inverse synthesis - recovering the
parameters that produce a given sound (Sections 1.1, 2 and 2.3) - and scores
sounds with a multi-scale spectrogram L1 distance (Section 4).  Two
estimators are built here, both counted in renders per target:

* gradient matching: a starting estimate (the learned proposal, or a random
  draw) followed by `steps` Adam steps on the logits z of u = sigmoid(z),
  each step one render, one MR-STFT loss and gradient, and one render
  adjoint, best-so-far tracked on the GPU (steps + 1 renders in all);
* random search: `budget` random parameter draws per target, best kept.

`MatchService` admits queued requests (targets of mixed lengths) into
batches of one length while the batch's device memory fits a byte budget,
runs gradient matching on each batch and reports per-request latency.

Orchestration only: rendering, the loss and its gradient, the adjoint, the
logit-space Adam step, the proposal and the best-so-far bookkeeping all run in
libsynth.so's kernels.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field

import numpy as np
import torch

from . import (NUM_PARAMS, synth_mrstft_loss, synth_mrstft_target, synth_mrstft_workspace,
               synth_render, synth_render_backward, synth_render_backward_workspace,
               synth_sample_params)
from . import learned as Lr

F32, F64 = torch.float32, torch.float64


@dataclass
class MatchResult:
    best_u: torch.Tensor          # float32 [T, 78]
    best_loss: torch.Tensor       # float64 [T] (MR-STFT L1 of the best render)
    best_step: torch.Tensor       # int64 [T]: render index (0 = the starting estimate)
    curve: list = field(default_factory=list)   # best-so-far mean loss after each render
    renders: int = 0
    snapshots: dict = field(default_factory=dict)   # render count -> best parameters then


def gradient_match(targets: torch.Tensor, voice_ids: torch.Tensor, nebula_table, u0: torch.Tensor,
                   steps: int = 50, lr: float = 0.05, noise_seed: int = 22,
                   init_eps: float = 1e-4, record_curve: bool = True,
                   snapshot_at=()) -> MatchResult:
    """Adam on logits from u0 for `steps` steps against targets [T, N].

    Candidate renders use voice_ids for the noise counter and `noise_seed` as
    the noise key (a key different from the targets': their noise is not
    recoverable).  Returns the best render over the trajectory; `snapshot_at`
    (render counts) keeps a copy of the best parameters after that many
    renders in result.snapshots."""
    T, N = targets.shape
    dev = targets.device
    z, u = Lr.logit_init(u0.contiguous(), init_eps)
    m = torch.zeros_like(z)
    v = torch.zeros_like(z)
    x = torch.empty(T, N, dtype=F32, device=dev)
    best = torch.full((T,), math.inf, dtype=F64, device=dev)
    best_step = torch.full((T,), -1, dtype=torch.int64, device=dev)
    best_u = torch.empty(T, NUM_PARAMS, dtype=F32, device=dev)
    gp = torch.empty(T, NUM_PARAMS, dtype=F32, device=dev)
    ws = None
    ws_loss = synth_mrstft_workspace(T, N, grad=steps > 0)
    tc = synth_mrstft_target(targets)          # target spectra, once per match
    gx = torch.empty(T, N, dtype=F32, device=dev) if steps > 0 else None
    curve = []
    snaps = {}
    for s in range(steps + 1):
        synth_render(u, nebula_table, n_samples=N, voice_ids=voice_ids, noise_seed=noise_seed, out=x)
        last = s == steps
        if last:
            loss = synth_mrstft_loss(x, tc, workspace=ws_loss)
        else:
            loss, gx = synth_mrstft_loss(x, tc, grad=True, workspace=ws_loss, out_grad=gx)
        Lr.best_update(loss, T, 1, 1, 0, best, best_step, col_base=s, params=u, best_params=best_u)
        if record_curve:
            curve.append(Lr.sum_f64(best, 1.0 / T))
        if s + 1 in snapshot_at:
            snaps[s + 1] = best_u.clone()
        if last:
            break
        if ws is None:
            ws = synth_render_backward_workspace(nebula_table, T, N)
        synth_render_backward(u, gx, nebula_table, voice_ids=voice_ids, noise_seed=noise_seed,
                              out=gp, workspace=ws)
        Lr.logit_adam(z, u, gp, m, v, s + 1, lr=lr)
    return MatchResult(best_u, best, best_step, [float(c) for c in curve], steps + 1, snaps)


def random_search(targets: torch.Tensor, voice_ids: torch.Tensor, nebula_table, budget: int = 1000,
                  seed: int = 21, noise_seed: int = 22, record_at=(1, 10, 51, 100, 1000),
                  snapshot_at=()):
    """`budget` random draws per target; candidate k of target t is voice
    t_id * budget + k of the generator keyed by `seed`.  Returns
    (best_u, best_loss, {budget: mean best loss}) and, with `snapshot_at`,
    a fourth item {budget: copy of the best parameters after that many}."""
    T, N = targets.shape
    dev = targets.device
    best = torch.full((T,), math.inf, dtype=F64, device=dev)
    best_k = torch.full((T,), -1, dtype=torch.int64, device=dev)
    best_u = torch.empty(T, NUM_PARAMS, dtype=F32, device=dev)
    x = torch.empty(T, N, dtype=F32, device=dev)
    base = voice_ids.to(torch.int64) * budget
    ws_loss = synth_mrstft_workspace(T, N)
    tc = synth_mrstft_target(targets)
    curve = {}
    snaps = {}
    for k in range(budget):
        cid = base + k
        u = synth_sample_params(seed, voice_ids=cid)
        synth_render(u, nebula_table, n_samples=N, voice_ids=voice_ids, noise_seed=noise_seed, out=x)
        loss = synth_mrstft_loss(x, tc, workspace=ws_loss)
        Lr.best_update(loss, T, 1, 1, 0, best, best_k, col_base=k, params=u, best_params=best_u)
        if (k + 1) in record_at:
            curve[k + 1] = float(Lr.sum_f64(best, 1.0 / T))
        if (k + 1) in snapshot_at:
            snaps[k + 1] = best_u.clone()
    if snapshot_at:
        return best_u, best, curve, snaps
    return best_u, best, curve


def logmel_l1(a: torch.Tensor, b: torch.Tensor, logmel: Lr.LogMel) -> torch.Tensor:
    """Per-voice mean |log-mel(a) - log-mel(b)| over the 128 x 64 features
    (float64 [B]; evaluation metric)."""
    fa, fb = logmel(a), logmel(b)
    return Lr.diff_reduce(fa, fb, kind=0, axis=1, scale=1.0 / fa.shape[1])


# ---------------------------------------------------------------------------
# Service: admission by device-memory budget, batches of one length
# ---------------------------------------------------------------------------
@dataclass
class Request:
    rid: int
    voice_id: int
    audio: torch.Tensor          # float32 [N] on the device


class MatchService:
    """Gradient sound matching for queued requests.

    Requests are served in arrival order; a batch takes the oldest queued
    request and every later queued request of the same length while the
    batch's device memory stays within `budget_bytes` (and at most
    `max_batch`).  Memory per request of N samples: target, render and
    gradient audio (12 N bytes), the adjoint workspace (168 bytes per control
    sample), parameter state and the proposal's features."""

    def __init__(self, nebula_table, proposal: Lr.Proposal | None = None, steps: int = 50,
                 lr: float = 0.05, budget_bytes: int = 64 << 30, max_batch: int = 1024,
                 init_seed: int = 21, noise_seed: int = 22, concurrency: int = 4):
        self.table = nebula_table
        self.proposal = proposal
        self.steps, self.lr = steps, lr
        self.budget, self.max_batch = budget_bytes, max_batch
        self.init_seed, self.noise_seed = init_seed, noise_seed
        self.concurrency = max(1, int(concurrency))

    @staticmethod
    def request_bytes(n_samples: int, q: int = 100) -> int:
        j = (n_samples + q - 1) // q
        return 12 * n_samples + 168 * j + 12 * 4 * NUM_PARAMS + 8192 * 6 + 64 * 1032 * 2

    def admit(self, queue: list, budget: int | None = None) -> list:
        """Pop the next batch (same length, within budget - by default the
        whole budget) from queue."""
        n = queue[0].audio.numel()
        per = self.request_bytes(n)
        cap = max(1, min(self.max_batch, (self.budget if budget is None else budget) // per))
        batch, rest = [], []
        for r in queue:
            if len(batch) < cap and r.audio.numel() == n:
                batch.append(r)
            else:
                rest.append(r)
        queue[:] = rest
        return batch

    def initial_estimate(self, targets, ids):
        if self.proposal is not None:
            return self.proposal(targets)
        return synth_sample_params(self.init_seed, voice_ids=ids)

    def run(self, requests: list):
        """Serve every request; returns (results {rid: (best_u, loss)},
        latencies {rid: seconds from the start until its batch finished on the
        GPU}, batches).  Up to `concurrency` batches are in flight at once,
        each on a stream of its own and together within the memory budget:
        the host enqueues a batch's whole gradient descent without waiting, so
        batches of different lengths share the GPU.  Initial estimates (the
        proposal's buffers are shared) are computed on the caller's stream."""
        queue = list(requests)
        results, lat, batches = {}, {}, []
        main = torch.cuda.current_stream()
        streams = [torch.cuda.Stream() for _ in range(self.concurrency)]
        free = list(range(self.concurrency))
        inflight, done = [], []
        used = 0
        torch.cuda.synchronize()
        start = torch.cuda.Event(enable_timing=True)
        start.record(main)
        while queue or inflight:
            per = self.request_bytes(queue[0].audio.numel()) if queue else 0
            if queue and free and (self.budget - used >= per or not inflight):
                batch = self.admit(queue, max(self.budget - used, per))
                n = batch[0].audio.numel()
                targets = torch.stack([r.audio for r in batch]).contiguous()
                # pinned host memory and an asynchronous copy: a copy from
                # pageable memory would wait for the batches in flight
                ids = torch.tensor([r.voice_id for r in batch], dtype=torch.int64).pin_memory()
                ids = ids.to(targets.device, non_blocking=True)
                u0 = self.initial_estimate(targets, ids).clone()
                k = free.pop(0)
                stream = streams[k]
                stream.wait_stream(main)
                with torch.cuda.stream(stream):
                    res = gradient_match(targets, ids, self.table, u0, steps=self.steps,
                                         lr=self.lr, noise_seed=self.noise_seed,
                                         record_curve=False)
                    end = torch.cuda.Event(enable_timing=True)
                    end.record(stream)
                for t in (targets, ids, u0):
                    t.record_stream(stream)
                nbytes = self.request_bytes(n) * len(batch)
                used += nbytes
                inflight.append((batch, n, nbytes, k, end, res))
            else:
                batch, n, nbytes, k, end, res = inflight.pop(0)   # the oldest batch
                end.synchronize()
                used -= nbytes
                free.append(k)
                done.append((batch, n, end, res))
        torch.cuda.synchronize()
        for batch, n, end, res in done:
            t = start.elapsed_time(end) / 1e3
            for i, r in enumerate(batch):
                results[r.rid] = (res.best_u[i], float(res.best_loss[i]))
                lat[r.rid] = t
            batches.append((len(batch), n, t))
        return results, lat, batches


def percentile(values, p):
    return float(np.percentile(np.asarray(list(values), dtype=np.float64), p))
