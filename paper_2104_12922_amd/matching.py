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


def gradient_match(targets: torch.Tensor, voice_ids: torch.Tensor, nebula_table, u0: torch.Tensor,
                   steps: int = 50, lr: float = 0.05, noise_seed: int = 22,
                   init_eps: float = 1e-4, record_curve: bool = True) -> MatchResult:
    """Adam on logits from u0 for `steps` steps against targets [T, N].

    Candidate renders use voice_ids for the noise counter and `noise_seed` as
    the noise key (a key different from the targets': their noise is not
    recoverable).  Returns the best render over the trajectory."""
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
    for s in range(steps + 1):
        synth_render(u, nebula_table, n_samples=N, voice_ids=voice_ids, noise_seed=noise_seed, out=x)
        last = s == steps
        if last:
            loss = synth_mrstft_loss(x, tc, workspace=ws_loss)
        else:
            loss, gx = synth_mrstft_loss(x, tc, grad=True, workspace=ws_loss, out_grad=gx)
        Lr.best_update(loss, T, 1, 1, 0, best, best_step, col_base=s, params=u, best_params=best_u)
        if record_curve:
            curve.append(best.mean())
        if last:
            break
        if ws is None:
            ws = synth_render_backward_workspace(nebula_table, T, N)
        synth_render_backward(u, gx, nebula_table, voice_ids=voice_ids, noise_seed=noise_seed,
                              out=gp, workspace=ws)
        Lr.logit_adam(z, u, gp, m, v, s + 1, lr=lr)
    return MatchResult(best_u, best, best_step, [float(c) for c in curve], steps + 1)


def random_search(targets: torch.Tensor, voice_ids: torch.Tensor, nebula_table, budget: int = 1000,
                  seed: int = 21, noise_seed: int = 22, record_at=(1, 10, 51, 100, 1000)):
    """`budget` random draws per target; candidate k of target t is voice
    t_id * budget + k of the generator keyed by `seed`.  Returns
    (best_u, best_loss, {budget: mean best loss})."""
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
    for k in range(budget):
        cid = base + k
        u = synth_sample_params(seed, voice_ids=cid)
        synth_render(u, nebula_table, n_samples=N, voice_ids=voice_ids, noise_seed=noise_seed, out=x)
        loss = synth_mrstft_loss(x, tc, workspace=ws_loss)
        Lr.best_update(loss, T, 1, 1, 0, best, best_k, col_base=k, params=u, best_params=best_u)
        if (k + 1) in record_at:
            curve[k + 1] = float(best.mean())
    return best_u, best, curve


def logmel_l1(a: torch.Tensor, b: torch.Tensor, logmel: Lr.LogMel) -> torch.Tensor:
    """Per-voice mean |log-mel(a) - log-mel(b)| (evaluation metric)."""
    return (logmel(a) - logmel(b)).abs().mean(dim=1)


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
                ids = torch.tensor([r.voice_id for r in batch], dtype=torch.int64,
                                   device=targets.device)
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


# ---------------------------------------------------------------------------
# Experiment: proposal + gradient matching vs random search
# ---------------------------------------------------------------------------
def _targets(table, first, count, seconds, seed):
    from . import synth_render, synth_sample_params
    ids = torch.arange(first, first + count, dtype=torch.int64, device="cuda")
    u = synth_sample_params(seed, voice_ids=ids)
    x = synth_render(u, table, n_samples=int(round(seconds * 44100)), voice_ids=ids, noise_seed=seed)
    return ids, x


def main(argv=None):
    """Train the proposal, then match targets of 1-4 s (length 1 + g mod 4 s)
    with the proposal + gradient steps, with random init + gradient steps, and
    by random search; print one JSON line of errors per render budget,
    throughput and service latency."""
    import argparse
    import json

    import workloads as W
    ap = argparse.ArgumentParser(description=main.__doc__)
    ap.add_argument("--targets", type=int, default=4096)
    ap.add_argument("--train-steps", type=int, default=2000)
    ap.add_argument("--train-batch", type=int, default=4096)
    ap.add_argument("--steps", type=int, default=50)
    ap.add_argument("--lr", type=float, default=0.05)
    ap.add_argument("--rs-budget", type=int, default=1000)
    ap.add_argument("--rs-targets", type=int, default=0, help="targets given to random search (0 = all)")
    ap.add_argument("--budget-gb", type=float, default=64.0)
    ap.add_argument("--concurrency", type=int, default=4,
                    help="matching batches in flight at once (one stream each)")
    a = ap.parse_args(argv)
    tab = W.default_nebula().table()
    out = {"targets": a.targets, "steps": a.steps, "lr": a.lr}

    t0 = time.perf_counter()
    prop, hist = Lr.train_proposal(tab, a.train_steps, batch=a.train_batch, seed=W.SEED_TRAIN,
                                   log_every=max(1, a.train_steps // 20),
                                   log=lambda s: print(s, flush=True))
    torch.cuda.synchronize()
    out["train"] = {"steps": a.train_steps, "batch": a.train_batch,
                    "seconds": time.perf_counter() - t0, "first_loss": hist[0][1],
                    "last_loss": hist[-1][1],
                    "heldout_mse": Lr.heldout_mse(prop, tab, seed=W.SEED_HELDOUT)}
    print(json.dumps({"train": out["train"]}), flush=True)

    lm = Lr.LogMel()
    budgets = sorted({1, 10, a.steps + 1, 100, a.rs_budget} & set(range(1, a.rs_budget + 1)))
    agg = {"proposal+gd": {}, "random+gd": {}, "random_search": {}, "logmel_l1": {}}
    counts = {}
    for secs in (1, 2, 3, 4):
        g = [i for i in range(a.targets) if 1 + i % 4 == secs]
        if not g:
            continue
        # targets of this length are the voices g = secs - 1, secs + 3, ... rendered at seed 20
        ids = torch.tensor(g, dtype=torch.int64, device="cuda")
        u = synth_sample_params(W.SEED_MATCH, voice_ids=ids)
        x = synth_render(u, tab, n_samples=secs * 44100, voice_ids=ids, noise_seed=W.SEED_MATCH)
        counts[secs] = len(g)
        r_p = gradient_match(x, ids, tab, prop(x), steps=a.steps, lr=a.lr)
        r_r = gradient_match(x, ids, tab, synth_sample_params(W.SEED_RS, voice_ids=ids),
                             steps=a.steps, lr=a.lr)
        nrs = len(g) if a.rs_targets == 0 else max(1, (a.rs_targets * len(g)) // a.targets)
        _, _, rs_curve = random_search(x[:nrs].contiguous(), ids[:nrs], tab, budget=a.rs_budget,
                                       record_at=tuple(budgets))
        for name, r in (("proposal+gd", r_p), ("random+gd", r_r)):
            for b in budgets:
                if b <= len(r.curve):
                    agg[name].setdefault(b, []).append((r.curve[b - 1], len(g)))
        for b, v in rs_curve.items():
            agg["random_search"].setdefault(b, []).append((v, nrs))
        y = synth_render(r_p.best_u, tab, n_samples=secs * 44100, voice_ids=ids, noise_seed=22)
        agg["logmel_l1"].setdefault("proposal+gd", []).append((float(logmel_l1(y, x, lm).mean()), len(g)))
        print(json.dumps({"seconds": secs, "n": len(g), "proposal+gd": r_p.curve[-1],
                          "random+gd": r_r.curve[-1], "random_search": rs_curve}), flush=True)

    def wmean(v):
        return sum(a * n for a, n in v) / sum(n for _, n in v)
    out["mrstft_l1_by_renders"] = {k: {str(b): wmean(v) for b, v in d.items()}
                                   for k, d in agg.items() if k != "logmel_l1"}
    out["logmel_l1"] = {k: wmean(v) for k, v in agg["logmel_l1"].items()}

    # service: requests in a fixed shuffled order, admission by memory budget
    order = np.random.default_rng(W.SEED_MATCH).permutation(a.targets)
    reqs = []
    for secs in (1, 2, 3, 4):
        g = [i for i in range(a.targets) if 1 + i % 4 == secs]
        if g:
            ids = torch.tensor(g, dtype=torch.int64, device="cuda")
            u = synth_sample_params(W.SEED_MATCH, voice_ids=ids)
            x = synth_render(u, tab, n_samples=secs * 44100, voice_ids=ids, noise_seed=W.SEED_MATCH)
            reqs += [Request(i, i, x[j]) for j, i in enumerate(g)]
    pos = {int(r): k for k, r in enumerate(order)}
    reqs.sort(key=lambda r: pos[r.rid])
    svc = MatchService(tab, prop, steps=a.steps, lr=a.lr, budget_bytes=int(a.budget_gb * 2**30),
                       concurrency=a.concurrency)
    t1 = time.perf_counter()
    _, lat, batches = svc.run(reqs)
    wall = time.perf_counter() - t1
    out["service"] = {"wall_s": wall, "requests_per_s": len(reqs) / wall,
                      "p50_s": percentile(lat.values(), 50), "p99_s": percentile(lat.values(), 99),
                      "batches": len(batches), "budget_gb": a.budget_gb,
                      "concurrency": a.concurrency,
                      "renders_per_request": a.steps + 1}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
