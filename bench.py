#!/usr/bin/env python3
"""Throughput of batched voice rendering on one MI355X.

Workload: 16384 voices of the default Voice, render lengths 1, 2 and 4 s
(by voice index mod 3) at 44.1 kHz packed back to back (1.686e9 samples,
6.74 GB of float32 audio), note durations uniform in [0.1, 4] s.  A step is
one pass of the hot path over the batch: the parameter draw (Philox) and the
fused render, with every input resident in HBM before the timed region.

Prints one JSON line: rendered samples/s (and MHz, x real time), the render
kernel's HBM roofline fraction (algorithmic bytes over its average launch time,
measured with HIP events on its stream; its VALU issue rate beside it), and
the float64 CPU oracle timed on a bounded sample of the same workload.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
# VALU issue peak: 256 CUs x 4 SIMDs x 16 lanes x 2.4 GHz lane-operations per
# second (a wave64 instruction occupies a SIMD for 4 cycles; transcendentals
# issue at half rate and count as 2)
VALU_PEAK_TOPS = 256 * 4 * 16 * 2.4e9 / 1e12
# minimum VALU lane-slots per output sample of the method as formulated: per
# computed sample about 43 (two float64 phase and increment updates 4, the
# sine's conversion and hardware sine 3, the square-saw's half-cycle reduction
# 4, sign flips 4, sine and cosine 4, tanh 7, shape 2, two VCA ramps and the mix
# 4, one eighth of a Philox-4x32-10 call 7.5 and the noise map and VCA 4),
# times the about 88% of output samples that precede the silent tails
RENDER_SLOTS_PER_SAMPLE = 38.0

# HBM bytes moved by one render launch on the ragged 16384-voice workload,
# from two rocprofv3 --pmc runs (FETCH_SIZE x 2.0 + WRITE_SIZE x 1.0 KiB; the
# factors make each counter read 1 GiB for a plain 1 GiB device copy).  Valid
# only for the kernel sources with this digest; reported as null otherwise.
RENDER_TRAFFIC = {"sources_sha256_16": "50789e57c17d3a78",
                  "fetch_bytes": 10880320, "write_bytes": 6758691344, "valu_busy": 0.91}
RENDER_SOURCES = ("render.hip", "voice_device.h", "philox.h", "series_tables.h")


def render_traffic():
    import hashlib
    h = hashlib.sha256()
    for f in RENDER_SOURCES:
        with open(os.path.join(ROOT, "paper_2104_12922_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    if h.hexdigest()[:16] != RENDER_TRAFFIC["sources_sha256_16"]:
        return None
    return RENDER_TRAFFIC


def parse():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--batch", type=int, default=16384)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=12.0)
    ap.add_argument("--graph", type=int, default=1, help="capture the step in a HIP graph")
    ap.add_argument("--rps", type=int, default=0, help="runs per segment (0 = library default)")
    ap.add_argument("--slices", type=int, default=0,
                    help="plain workload: slices per voice with chunk carries (0 = library default)")
    ap.add_argument("--autotune", type=int, default=1,
                    help="time the candidate launch plans on this batch first (untimed) and "
                         "render with the fastest")
    ap.add_argument("--no-match", action="store_true",
                    help="leave the sound-matching experiment out of the headline line")
    ap.add_argument("--match-targets", type=int, default=4096)
    ap.add_argument("--match-train-steps", type=int, default=12208)
    ap.add_argument("--workload", default="render",
                    choices=("render", "plain", "learned", "grad", "match", "nebula", "vcf", "fm"),
                    help="render: the headline ragged render; plain: 128 voices x 4 s "
                         "(200 renders per timed step, in a HIP graph); learned: one proposal "
                         "training step (render + log-mel + MLP); grad: render, MR-STFT "
                         "loss and gradient, render adjoint; match: the sound-matching "
                         "experiment alone; nebula: MMD of 1000 x 1000 log-mel sets and "
                         "nebula-search trials (256 sounds x 4 s each); vcf: the resonant "
                         "low-pass filter and its adjoint on the ragged 16384-voice renders; "
                         "fm: the 4-operator FM voice on the ragged 16384-voice batch")
    ap.add_argument("--copy-bytes", type=int, default=0,
                    help="only run a plain device-to-device copy of this many bytes (the "
                         "reference point that scales HBM byte counters) and exit")
    return ap.parse_args()


def copy_only(nbytes):
    """A plain copy kernel of known size: reads and writes nbytes once each."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    torch.cuda.synchronize()
    ev = _events(3)
    for a, b in ev:
        a.record()
        dst.copy_(src)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev[1:]]))
    print(json.dumps({"copy_bytes": nbytes, "launches": 3, "ms_per_copy": ms,
                      "read_plus_write_GBps": 2.0 * nbytes / (ms * 1e-3) / 1e9}), flush=True)


def cpu_baseline(wl, min_seconds):
    """Float64 oracle on consecutive 128-voice batches of the workload (mixed
    1/2/4 s lengths) until at least min_seconds of CPU wall time are spent."""
    import torch
    from oracle import philox, voice
    threads = len(os.sched_getaffinity(0))
    torch.set_num_threads(threads)
    n = 0
    v0 = 0
    dt = 0.0
    while dt < min_seconds and v0 < wl.batch:
        ids = np.arange(v0, min(v0 + 128, wl.batch))
        u = philox.sample_params(wl.seed, ids)
        t0 = time.perf_counter()
        y = voice.render(torch.from_numpy(u), ids, wl.lengths[ids], wl.nebula.table(),
                         wl.sample_rate, wl.control_rate, wl.key_noise())
        dt += time.perf_counter() - t0
        assert y.numel() == int(wl.lengths[ids].sum())
        n += y.numel()
        v0 = int(ids[-1]) + 1
        del y
    return {"value": n / dt, "unit": "samples/s", "cores": threads, "kind": "oracle",
            "sample": f"float64 oracle render of voices 0..{v0 - 1} of the workload "
                      f"({n} samples, 1/2/4 s mix) in batches of 128, {dt:.1f} s wall"}


def _events(n):
    import torch
    return [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
            for _ in range(n)]


def bench_learned(args):
    """One training step of the proposal at batch 4096: draw and render 4096
    training voices (1-4 s by voice index mod 4), log-mel features of the
    64 frames, standardisation, MLP forward + backward + Adam.  Per-phase
    times come from steps run one after another; `value` from the training
    loop, which overlaps the render of step s + 1 with the MLP of step s."""
    import torch
    import workloads as W
    from paper_2104_12922_amd import learned as Lr
    B = 4096
    tab = W.default_nebula().table()
    lm = Lr.LogMel()
    net = Lr.MLP(W.mlp_init(0))
    stream = torch.cuda.Stream()
    mlp_flop = 2.0 * (8192 * 1024 + 1024 * 1024 + 1024 * 78) * 3 - 2.0 * 8192 * 1024
    with torch.cuda.stream(stream):
        ids = Lr.train_ids(0, B)
        u, audio, offs = Lr.render_batch(W.SEED_TRAIN, ids, tab)
        feat = lm(audio, offsets=offs)
        mean, inv_std = Lr.feature_stats(feat)
        x = Lr.standardize(feat, mean, inv_std)
        torch.cuda.synchronize()
        n_ev = max(1, min(args.steps, 10))
        e_r, e_l, e_m = _events(n_ev), _events(n_ev), _events(n_ev)
        t_step = []
        for i in range(args.warmup + args.steps):
            first = (i + 1) * B
            t0 = time.perf_counter()
            j = i - args.warmup
            if 0 <= j < n_ev:
                e_r[j][0].record(stream)
            ids = Lr.train_ids(first, B)
            u, audio, offs = Lr.render_batch(W.SEED_TRAIN, ids, tab)
            if 0 <= j < n_ev:
                e_r[j][1].record(stream)
                e_l[j][0].record(stream)
            lm(audio, out=feat, offsets=offs)
            if 0 <= j < n_ev:
                e_l[j][1].record(stream)
                e_m[j][0].record(stream)
            Lr.standardize(feat, mean, inv_std, out=x)
            net.train_step(x, u)
            if 0 <= j < n_ev:
                e_m[j][1].record(stream)
            torch.cuda.synchronize()
            if j >= 0:
                t_step.append(time.perf_counter() - t0)
        ms = lambda ev: float(np.mean([a.elapsed_time(b) for a, b in ev]))
        r_ms, l_ms, m_ms = ms(e_r), ms(e_l), ms(e_m)
        # the training loop proper overlaps consecutive steps: the render,
        # log-mel and standardisation of step s + 1 on this stream, the MLP
        # of step s on a second one (Lr.train_pipelined); K steps timed
        first = args.warmup + args.steps + 1
        Lr.train_pipelined(net, lm, tab, mean, inv_std, args.warmup, B, W.SEED_TRAIN,
                           first=first)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        Lr.train_pipelined(net, lm, tab, mean, inv_std, args.steps, B, W.SEED_TRAIN,
                           first=first + args.warmup)
        torch.cuda.synchronize()
        pipe_s = (time.perf_counter() - t0) / args.steps
    step_s = float(np.mean(t_step))
    # log-mel algorithmic bytes (one fused kernel): frame samples inside each
    # voice read once (float32; frames do not overlap at hop 2756), the
    # float32 features written
    lens = np.array([int(round(s * 44100.0)) for s in (1, 2, 3, 4)])[np.arange(B) % 4]
    inside = int(np.clip(lens[:, None] - 2756 * np.arange(64)[None, :], 0, 2048).sum())
    mel_bytes = 4.0 * inside + 4.0 * B * 8192
    gbs = mel_bytes / (l_ms * 1e-3) / 1e9
    out = {"metric": "proposal training voices/sec", "value": B / pipe_s, "unit": "voices/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": pipe_s * 1e3,
           "serial_ms_per_step": step_s * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic (Philox-drawn training voices rendered on the fly)",
           "config": {"workload": "proposal_train_b4096_1-4s", "batch": B,
                      "features": "log-mel 128 x 64 (FFT power spectrum)",
                      "mlp": "8192-1024-1024-78"},
           "phase_ms": {"render": r_ms, "logmel": l_ms, "mlp_train": m_ms},
           "render_plans": (dict(Lr._TUNER.table) if Lr._TUNER is not None else None),
           "render_plan_ms": (dict(Lr._TUNER.timings) if Lr._TUNER is not None else None),
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "logmel_fft_kernel (FFT, power, mel bands, log)",
                        "alg_bytes_per_launch": mel_bytes},
           "mlp_tflops": mlp_flop * B / (m_ms * 1e-3) / 1e12}
    print(json.dumps(out), flush=True)


def bench_plain(args):
    """The plain render: 128 voices x 4 s (22.6 M samples).  One render takes
    tens of microseconds, so a timed step is 200 back-to-back renders captured
    in one HIP graph; value = rendered samples per second."""
    import torch
    import workloads as W
    import paper_2104_12922_amd as S
    wl = W.plain_render()
    tab = wl.nebula.table()
    B, N = wl.batch, 176400
    stream = torch.cuda.Stream()
    reps = 200
    with torch.cuda.stream(stream):
        u = S.synth_sample_params(wl.seed, 0, B)
        out = torch.empty(B, N, device="cuda")
        if args.slices:                 # an explicit plan: slices per voice, chunk carries first
            rps = args.rps or 4
            import ctypes
            from paper_2104_12922_amd import _native
            cfg, keep = _native.make_config(tab)
            need = _native.lib().synth_render_plan_workspace(ctypes.byref(cfg), B, N)
            ws = torch.empty(max(1, need), dtype=torch.uint8, device="cuda")

            def render():
                S.synth_render_plan(u, tab, rps, args.slices, n_samples=N,
                                    noise_seed=wl.key_noise(), out=out, carries=True, workspace=ws)
        else:                           # the library's default plan

            def render():
                S.synth_render(u, tab, n_samples=N, noise_seed=wl.key_noise(), out=out)
        render()
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for _ in range(reps):
                render()
        torch.cuda.synchronize()
        for _ in range(args.warmup):
            g.replay()
        torch.cuda.synchronize()
        ts = []
        for _ in range(args.steps):
            a, b = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
            a.record(stream)
            g.replay()
            b.record(stream)
            b.synchronize()
            ts.append(a.elapsed_time(b))
    ms = float(np.mean(ts))
    per = ms / reps
    alg = 4.0 * B * N + 312.0 * B
    out = {"metric": "rendered audio samples/sec", "value": B * N / (per * 1e-3),
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": ms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl.name, "voices": B, "samples": B * N,
                      "renders_per_step": reps,
                      "plan": {"rps": args.rps or 4, "slices": args.slices} if args.slices
                      else "library default"},
           "roofline": {"bound": "hbm", "achieved": alg / (per * 1e-3) / 1e9,
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": alg / (per * 1e-3) / 1e9 / HBM_PEAK_GBS, "traffic": None,
                        "kernel": "render_kernel", "kernel_ms": per}}
    print(json.dumps(out), flush=True)


def bench_grad(args):
    """Gradient workload: 256 voices x 4 s rendered, MR-STFT loss and gradient
    against targets of another seed, render adjoint to the 78 parameters."""
    import torch
    import workloads as W
    import paper_2104_12922_amd as S
    wl = W.gradient_batch()
    tab = wl.nebula.table()
    B, N = wl.batch, 176400
    stream = torch.cuda.Stream()
    with torch.cuda.stream(stream):
        u = S.synth_sample_params(wl.seed, 0, B)
        ut = S.synth_sample_params(W.SEED_TARGET, 0, B)
        t = S.synth_render(ut, tab, n_samples=N, noise_seed=W.SEED_TARGET)
        x = torch.empty(B, N, device="cuda")
        gp = torch.empty(B, 78, device="cuda")
        ws = S.synth_render_backward_workspace(tab, B, N)
        ws_loss = S.synth_mrstft_workspace(B, N, grad=True)
        tc = S.synth_mrstft_target(t)            # the target's spectra, computed once
        gx = torch.empty(B, N, device="cuda")
        n_ev = max(1, min(args.steps, 10))
        e = [_events(n_ev) for _ in range(3)]
        tt = []
        for i in range(args.warmup + args.steps):
            j = i - args.warmup
            t0 = time.perf_counter()
            if 0 <= j < n_ev:
                e[0][j][0].record(stream)
            S.synth_render(u, tab, n_samples=N, noise_seed=wl.seed, out=x)
            if 0 <= j < n_ev:
                e[0][j][1].record(stream)
                e[1][j][0].record(stream)
            loss, gx = S.synth_mrstft_loss(x, tc, grad=True, workspace=ws_loss, out_grad=gx)
            if 0 <= j < n_ev:
                e[1][j][1].record(stream)
                e[2][j][0].record(stream)
            S.synth_render_backward(u, gx, tab, noise_seed=wl.seed, workspace=ws, out=gp)
            if 0 <= j < n_ev:
                e[2][j][1].record(stream)
            torch.cuda.synchronize()
            if j >= 0:
                tt.append(time.perf_counter() - t0)
        ms = [float(np.mean([a.elapsed_time(b) for a, b in ev])) for ev in e]
    step = float(np.mean(tt))
    out = {"metric": "gradient steps voices/sec", "value": B / step, "unit": "voices/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": step * 1e3,
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
           "data": "synthetic", "config": {"workload": wl.name, "voices": B, "samples": B * N},
           "phase_ms": {"render": ms[0], "mrstft_loss_grad": ms[1], "render_adjoint": ms[2]}}
    print(json.dumps(out), flush=True)


def bench_nebula(args):
    """MMD between two sets of 1000 sounds' log-mel embeddings (8192 floats;
    the paper's trial size) with its VALU roofline, and the rate of nebula
    search trials (draw, render, embed 256 sounds of 4 s, MMD against 256
    target sounds)."""
    import torch
    import workloads as W
    from paper_2104_12922_amd import nebula as NB
    n, dim = 1000, 8192
    g = torch.Generator().manual_seed(0)
    X = (torch.randn(n, dim, generator=g) - 4.0).cuda()
    Y = (torch.randn(n, dim, generator=g) * 1.1 - 4.0).cuda()
    out = torch.empty(4, dtype=torch.float64, device="cuda")
    ws = NB._Workspace()
    for _ in range(max(1, args.warmup)):
        NB.mmd_l1(X, Y, out=out, workspace=ws)
    torch.cuda.synchronize()
    ev = _events(args.steps)
    for a, b in ev:
        a.record()
        NB.mmd_l1(X, Y, out=out, workspace=ws)
        b.record()
    torch.cuda.synchronize()
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    pair_dims = 3.0 * n * n * dim            # S(X, Y), S(X, X), S(Y, Y)
    tops = 2.0 * pair_dims / (ms * 1e-3) / 1e12
    # search trials: 256 sounds x 4 s from the default nebula with random curves
    base = W.default_nebula().table()
    sets = NB.SoundSets(n_sounds=256, n_samples=176400, seed=30)
    target = sets.embed(base, 10 ** 6).clone()
    search = NB.NebulaSearch(base, target, sets=sets, target_per_trial=256, seed=1)
    rng = np.random.default_rng(0)
    trials = max(4, args.steps)
    for k in range(2):
        search.score(rng.uniform(-1, 1, 78), k)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(trials):
        search.score(rng.uniform(-1, 1, 78), 2 + k)
    torch.cuda.synchronize()
    trial_s = (time.perf_counter() - t0) / trials
    res = {"metric": "MMD pair sums and nebula-search trials", "value": 1.0 / trial_s,
           "unit": "trials/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": trial_s * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": "mmd_1000x1000_logmel8192 + search trial 256 x 4 s",
                      "mmd_sets": [n, n], "dim": dim, "trial_sounds": 256, "trial_target": 256},
           "mmd_ms": ms, "mmd": float(out[0]),
           "roofline": {"bound": "alu", "achieved": tops, "peak": VALU_PEAK_TOPS,
                        "unit": "T VALU lane-slots/s", "frac": tops / VALU_PEAK_TOPS,
                        "traffic": None, "kernel": "l1_pair_sum_kernel",
                        "alg_slots_per_launch_set": 2.0 * pair_dims}}
    print(json.dumps(res), flush=True)


def bench_vcf(args):
    """Resonant low-pass filter (forward and adjoint) on the rendered ragged
    16384-voice batch (1, 2 and 4 s voices), cutoff driven by a control-rate
    envelope per voice."""
    import torch
    import workloads as W
    import paper_2104_12922_amd as S
    from paper_2104_12922_amd import vcf as V
    wl = W.ragged_batch(args.batch)
    B = wl.batch
    offs = torch.from_numpy(wl.offsets).cuda()
    lmax = int(wl.lengths.max())
    u = S.synth_sample_params(wl.seed, 0, B)
    x = S.synth_render(u, wl.nebula.table(), offsets=offs, noise_seed=wl.key_noise())
    gen = torch.Generator(device="cuda").manual_seed(0)
    J = (lmax + 99) // 100
    env = torch.rand(B, J, device="cuda", generator=gen)
    params = torch.stack([torch.rand(B, device="cuda", generator=gen) * 70 + 30,
                          torch.rand(B, device="cuda", generator=gen) * 72 - 24,
                          torch.rand(B, device="cuda", generator=gen) * 14.5 + 0.5], 1).contiguous()
    g = torch.randn(x.numel(), device="cuda", generator=gen)
    y = torch.empty_like(x)
    # launch order: longest voices first (lengths known with the batch)
    order = torch.from_numpy(np.argsort(-wl.lengths, kind="stable").astype(np.int32)).cuda()
    for _ in range(max(1, args.warmup)):
        _, st = V.lowpass(x, env, params, 100, offsets=offs, max_samples=lmax, keep_states=True,
                          out=y, order=order)
        V.lowpass_backward(x, g, env, params, st, 100, offsets=offs, max_samples=lmax, order=order)
    torch.cuda.synchronize()
    ef, eb = _events(args.steps), _events(args.steps)
    for i in range(args.steps):
        ef[i][0].record()
        _, st = V.lowpass(x, env, params, 100, offsets=offs, max_samples=lmax, keep_states=True,
                          out=y, order=order)
        ef[i][1].record()
        eb[i][0].record()
        V.lowpass_backward(x, g, env, params, st, 100, offsets=offs, max_samples=lmax, order=order)
        eb[i][1].record()
    torch.cuda.synchronize()
    fms = float(np.mean([a.elapsed_time(b) for a, b in ef]))
    bms = float(np.mean([a.elapsed_time(b) for a, b in eb]))
    n = x.numel()
    fgbs, bgbs = 8.0 * n / (fms * 1e-3) / 1e9, 12.0 * n / (bms * 1e-3) / 1e9
    res = {"metric": "filtered audio samples/sec (forward + adjoint)", "value": n / ((fms + bms) * 1e-3),
           "unit": "samples/s", "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
           "ms_per_step": fms + bms, "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
           "dtype": "f64", "data": "synthetic",
           "config": {"workload": wl.name, "voices": B, "samples": n, "period": 100,
                      "launch_order": "longest voices first"},
           "forward_ms": fms, "adjoint_ms": bms,
           "roofline": {"bound": "hbm", "achieved": fgbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": fgbs / HBM_PEAK_GBS, "traffic": None, "kernel": "vcf_forward_kernel",
                        "alg_bytes_per_launch": 8.0 * n},
           "adjoint_roofline": {"bound": "hbm", "achieved": bgbs, "peak": HBM_PEAK_GBS,
                                "unit": "GB/s", "frac": bgbs / HBM_PEAK_GBS,
                                "kernel": "vcf_backward_kernel", "alg_bytes_per_launch": 12.0 * n}}
    print(json.dumps(res), flush=True)


def bench_fm(args):
    """The 4-operator FM voice: parameter draw and render of the ragged
    16384-voice batch (1, 2 and 4 s voices, note durations 0.1-4 s)."""
    import torch
    import workloads as W
    from paper_2104_12922_amd import fm as FMV
    wl = W.ragged_batch(args.batch)
    B = wl.batch
    offs = torch.from_numpy(wl.offsets).cuda()
    tab = W.fm_default_nebula(duration_min=0.1).table()
    out = torch.empty(wl.total_samples, dtype=torch.float32, device="cuda")
    order = torch.from_numpy(np.argsort(-wl.lengths, kind="stable").astype(np.int32)).cuda()
    for _ in range(max(1, args.warmup)):
        u = FMV.fm_sample_params(wl.seed, batch=B)
        FMV.fm_render(u, tab, offsets=offs, out=out, order=order)
    torch.cuda.synchronize()
    ev = _events(args.steps)
    t0 = time.perf_counter()
    for a, b in ev:
        a.record()
        u = FMV.fm_sample_params(wl.seed, batch=B)
        FMV.fm_render(u, tab, offsets=offs, out=out, order=order)
        b.record()
    torch.cuda.synchronize()
    wall = (time.perf_counter() - t0) / args.steps
    ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    n = wl.total_samples
    gbs = 4.0 * n / (ms * 1e-3) / 1e9
    res = {"metric": "rendered FM audio samples/sec", "value": n / (ms * 1e-3), "unit": "samples/s",
           "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
           "wall_ms_per_step": wall * 1e3, "higher_is_better": True, "scaling": "weak",
           "vs_baseline": None, "dtype": "f32", "data": "synthetic",
           "config": {"workload": wl.name + "_fm4", "voices": B, "samples": n,
                      "launch_order": "longest voices first"},
           "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": gbs / HBM_PEAK_GBS, "traffic": None, "kernel": "fm_render_kernel",
                        "alg_bytes_per_launch": 4.0 * n}}
    print(json.dumps(res), flush=True)


def sound_match(targets=4096, train_steps=12208, train_batch=4096, steps=50, lr=0.05,
                rs_budget=1000, budget_gb=64.0, concurrency=4, log=None):
    """Sound matching (the second half of the headline metric): train the
    learned proposal on 12208 x 4096 = 5e7 voices rendered on the fly (seed
    10), report its held-out parameter MSE and re-rendered log-mel L1 (seed
    11), then match targets of 1-4 s (length 1 + g mod 4 s, seed 20) three
    ways - proposal + 50 Adam steps through the adjoint, random start + 50
    steps (the no-MLP ablation), random search with 1000 draws (seed 21) -
    and report the mean MR-STFT L1 and log-mel L1 of the best render after
    1, 10, 51, 100 and 1000 renders per target; then serve the targets as
    queued requests (memory-budget admission) for p50/p99 latency."""
    import torch
    import workloads as W
    import paper_2104_12922_amd as S
    from paper_2104_12922_amd import learned as Lr, matching as M
    say = log or (lambda *a: None)
    tab = W.default_nebula().table()
    out = {"targets": targets, "adam_steps": steps, "lr": lr}
    t0 = time.perf_counter()
    prop, hist = Lr.train_proposal(tab, train_steps, init=W.mlp_init(0), batch=train_batch,
                                   seed=W.SEED_TRAIN)
    torch.cuda.synchronize()
    train_s = time.perf_counter() - t0
    per = Lr.heldout_mse(prop, tab, seed=W.SEED_HELDOUT, per_param=True)
    out["train"] = {"steps": train_steps, "batch": train_batch, "voices": train_steps * train_batch,
                    "seconds": train_s, "first_loss": hist[0][1],
                    "last_loss": hist[-1][1],
                    "heldout_param_mse": float(per.mean()),
                    "heldout_param_mse_predicting_half": 1.0 / 12.0,
                    # the two parameters a log-mel spectrogram determines best
                    "heldout_param_mse_pitch": float(per[0]),
                    "heldout_param_mse_duration": float(per[1]),
                    # parameters whose error is below half that of predicting 0.5
                    "params_below_half_of_predicting_half": int((per < 0.5 / 12.0).sum()),
                    "heldout_logmel_l1": Lr.heldout_logmel_l1(prop, tab, seed=W.SEED_HELDOUT)}
    say("sound_match train", out["train"])
    lm = Lr.LogMel()
    budgets = tuple(sorted({1, 10, steps + 1, 100, rs_budget}))
    acc = {}

    def add(method, b, mr, l1, n):
        a = acc.setdefault(method, {}).setdefault(b, [0.0, 0.0, 0])
        a[0] += mr * n
        a[1] += l1 * n
        a[2] += n

    for secs in (1, 2, 3, 4):
        g = [i for i in range(targets) if 1 + i % 4 == secs]
        if not g:
            continue
        ids = torch.tensor(g, dtype=torch.int64, device="cuda")
        n = secs * 44100
        x = S.synth_render(S.synth_sample_params(W.SEED_MATCH, voice_ids=ids), tab, n_samples=n,
                           voice_ids=ids, noise_seed=W.SEED_MATCH)

        def l1_of(u):
            y = S.synth_render(u, tab, n_samples=n, voice_ids=ids, noise_seed=W.SEED_CAND_NOISE)
            return float(Lr.sum_f64(M.logmel_l1(y, x, lm), 1.0 / len(g)))

        r_p = M.gradient_match(x, ids, tab, prop(x), steps=steps, lr=lr, snapshot_at=budgets)
        r_r = M.gradient_match(x, ids, tab, S.synth_sample_params(W.SEED_RS, voice_ids=ids),
                               steps=steps, lr=lr, snapshot_at=budgets)
        _, _, rs_curve, rs_snaps = M.random_search(x, ids, tab, budget=rs_budget, seed=W.SEED_RS,
                                                   record_at=budgets, snapshot_at=budgets)
        for name, r in (("proposal+gd", r_p), ("random_init+gd", r_r)):
            for b, u in r.snapshots.items():
                add(name, b, r.curve[b - 1], l1_of(u), len(g))
        for b, u in rs_snaps.items():
            add("random_search", b, rs_curve[b], l1_of(u), len(g))
        say("sound_match", secs, "s: proposal+gd", r_p.curve[-1], "random_init+gd", r_r.curve[-1],
            "random_search", rs_curve)
    out["mrstft_l1"] = {m: {str(b): v[0] / v[2] for b, v in sorted(d.items())} for m, d in acc.items()}
    out["logmel_l1"] = {m: {str(b): v[1] / v[2] for b, v in sorted(d.items())} for m, d in acc.items()}
    rs_best = out["mrstft_l1"]["random_search"][str(rs_budget)]
    reach = [int(b) for b, v in out["mrstft_l1"]["proposal+gd"].items() if v <= rs_best]
    out["renders_to_random_search_best"] = {
        "proposal+gd": min(reach) if reach else None, "random_search": rs_budget}

    # service: requests in a fixed shuffled order, admission by device-memory budget
    order = np.random.default_rng(W.SEED_MATCH).permutation(targets)
    reqs = []
    for secs in (1, 2, 3, 4):
        g = [i for i in range(targets) if 1 + i % 4 == secs]
        if g:
            ids = torch.tensor(g, dtype=torch.int64, device="cuda")
            x = S.synth_render(S.synth_sample_params(W.SEED_MATCH, voice_ids=ids), tab,
                               n_samples=secs * 44100, voice_ids=ids, noise_seed=W.SEED_MATCH)
            reqs += [M.Request(i, i, x[j]) for j, i in enumerate(g)]
    pos = {int(r): k for k, r in enumerate(order)}
    reqs.sort(key=lambda r: pos[r.rid])
    svc = M.MatchService(tab, prop, steps=steps, lr=lr, budget_bytes=int(budget_gb * 2**30),
                         concurrency=concurrency)
    t1 = time.perf_counter()
    _, lat, batches = svc.run(reqs)
    wall = time.perf_counter() - t1
    out["service"] = {"wall_s": wall, "requests_per_s": len(reqs) / wall,
                      "p50_s": M.percentile(lat.values(), 50), "p99_s": M.percentile(lat.values(), 99),
                      "batches": len(batches), "budget_gb": budget_gb, "concurrency": concurrency,
                      "renders_per_request": steps + 1}
    out["seconds"] = time.perf_counter() - t0
    return out


class RenderStep:
    """The timed step of the headline workload: the parameter draw and the
    ragged render of the whole batch, inputs resident in HBM, voices launched
    longest first, the launch plan autotuned on this batch (untimed).  The
    draw and the render are captured in two HIP graphs replayed back to back,
    so that HIP events between the two replays time the render kernel inside
    the timed steps.  ``run()`` performs one step; ``params`` and ``audio``
    hold its results."""

    def __init__(self, wl, rps=0, autotune=True, graph=True):
        import torch
        import paper_2104_12922_amd as S
        self.S, self.wl = S, wl
        self.table = wl.nebula.table()
        dev = torch.device("cuda:0")
        torch.cuda.set_device(dev)
        B = wl.batch
        self.offsets = torch.from_numpy(wl.offsets).to(dev)
        self.params = torch.empty(B, 78, dtype=torch.float32, device=dev)
        self.audio = torch.empty(wl.total_samples, dtype=torch.float32, device=dev)
        self.stream = torch.cuda.Stream(device=dev)
        # launch order: longest voices first (the lengths are known with the
        # offsets), so that short voices fill the end of the launch
        self.order = torch.from_numpy(np.argsort(-wl.lengths, kind="stable").astype(np.int32)).to(dev)
        self.lmax = int(wl.lengths.max())
        self.plan = (4, 1, 0, 0)                       # the library's default plan
        if rps:
            self.plan = (rps, 1, 0, 0)
        elif autotune:
            from paper_2104_12922_amd.autotune import RenderTuner
            with torch.cuda.stream(self.stream):
                self.draw()
                self.plan, _ = RenderTuner().tune(self.params, self.table, offsets=self.offsets,
                                                  order=self.order, max_samples=self.lmax,
                                                  noise_seed=wl.key_noise(), out=self.audio)
            torch.cuda.synchronize()
        self.graphs = None
        with torch.cuda.stream(self.stream):
            self.draw()
            self.render()
            torch.cuda.synchronize()
            if graph:
                self.graphs = (torch.cuda.CUDAGraph(), torch.cuda.CUDAGraph())
                with torch.cuda.graph(self.graphs[0], stream=self.stream):
                    self.draw()
                with torch.cuda.graph(self.graphs[1], stream=self.stream):
                    self.render()
                torch.cuda.synchronize()

    def draw(self):
        wl = self.wl
        self.S.synth_sample_params(wl.seed, wl.first_g, wl.batch, out=self.params)

    def render(self):
        p, wl = self.plan, self.wl
        self.S.synth_render_plan(self.params, self.table, p[0], p[1], persistent=bool(p[2]),
                                 grid_blocks=p[3], offsets=self.offsets,
                                 carries=len(p) > 4 and bool(p[4]), max_samples=self.lmax,
                                 order=self.order, noise_seed=wl.key_noise(), out=self.audio)

    def run(self, events=None):
        """One step; `events` (a pair of torch.cuda.Event) bracket the render."""
        import torch
        with torch.cuda.stream(self.stream):
            if self.graphs is not None:
                self.graphs[0].replay()
            else:
                self.draw()
            if events is not None:
                events[0].record(self.stream)
            if self.graphs is not None:
                self.graphs[1].replay()
            else:
                self.render()
            if events is not None:
                events[1].record(self.stream)


def main():
    args = parse()
    if args.gpus != 1:
        print(json.dumps({"error": "the renderer is benchmarked on one GPU only (voices shard with no communication); --gpus must be 1"}))
        sys.exit(2)
    if args.copy_bytes:
        copy_only(args.copy_bytes)
        return
    if args.workload == "learned":
        return bench_learned(args)
    if args.workload == "grad":
        return bench_grad(args)
    if args.workload == "plain":
        return bench_plain(args)
    if args.workload == "nebula":
        return bench_nebula(args)
    if args.workload == "vcf":
        return bench_vcf(args)
    if args.workload == "fm":
        return bench_fm(args)
    if args.workload == "match":
        res = sound_match(targets=args.match_targets, train_steps=args.match_train_steps,
                          log=lambda *a: print(*a, file=sys.stderr, flush=True))
        print(json.dumps({"metric": "sound-match MR-STFT and log-mel L1 per render budget",
                          "sound_match": res}), flush=True)
        return
    import torch
    import workloads as W

    wl = W.ragged_batch(args.batch)
    st = RenderStep(wl, rps=args.rps, autotune=bool(args.autotune), graph=bool(args.graph))
    # the render kernel's duration in every timed step: HIP events on its
    # stream, recorded between the draw and render graph replays
    ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
          for _ in range(args.steps)]
    for _ in range(args.warmup):
        st.run()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for k in range(args.steps):
        st.run(ev[k])
    torch.cuda.synchronize()
    dt = time.perf_counter() - t0
    kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))
    plan, B, total = st.plan, wl.batch, wl.total_samples

    prof = render_traffic() if wl.batch == 16384 and plan in (None, (4, 1, 0, 0)) else None
    ms = dt / args.steps * 1e3
    value = total / (dt / args.steps)
    alg_bytes = 4.0 * total + 4.0 * 78 * B + 8.0 * (B + 1) + 4.0 * B   # audio, params, offsets, order
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    alu_tops = RENDER_SLOTS_PER_SAMPLE * total / (kern_ms * 1e-3) / 1e12
    out = {
        # the headline metric: value is the render throughput; the sound-match
        # L1 per render budget is the "sound_match" object
        "metric": "rendered audio samples/sec (MHz, x real-time) & sound-match log-mel L1 per render budget",
        "value": value, "unit": "samples/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup, "ms_per_step": ms,
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "f32",
        "data": "synthetic (Philox-drawn parameters, rendered on the fly)",
        "config": {"workload": wl.name, "voices": B, "samples": total,
                   "lengths_s": [1, 2, 4], "sample_rate": wl.sample_rate,
                   "control_rate": wl.control_rate, "note_duration_s": [0.1, 4.0],
                   "hip_graph": bool(args.graph), "phase_dtype": "f64",
                   "launch_plan": list(plan) if plan is not None else "default",
                   "launch_order": "longest voices first"},
        "mhz": value / 1e6, "x_realtime": value / wl.sample_rate,
        # the HBM roofline of the render kernel: algorithmic bytes per launch
        # (4 B per output sample + 312 B of parameters, 8 B of offsets and 4 B
        # of launch order per voice) / its average launch time.  The kernel is
        # limited by VALU issue below that roofline; "alu" gives the issue rate
        # against a per-sample floor of this formulation's own count (a lower
        # bound counted for this design, not a hardware constant).
        "roofline": {"bound": "hbm", "achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": achieved / HBM_PEAK_GBS,
                     "traffic": (float(prof["fetch_bytes"] + prof["write_bytes"])
                                 if prof else None),
                     "alg_bytes_per_launch": alg_bytes,
                     "kernel": "render_kernel", "kernel_ms": kern_ms,
                     "alu": {"achieved": alu_tops, "peak": VALU_PEAK_TOPS,
                             "unit": "T VALU lane-slots/s", "frac": alu_tops / VALU_PEAK_TOPS,
                             "slots_per_sample_floor": RENDER_SLOTS_PER_SAMPLE,
                             "floor_basis": "this design's own count of issue slots per sample",
                             "valu_busy_profiled": prof["valu_busy"] if prof else None}},
        "context": {"paper_single_gpu_mhz": 714.0, "paper_gpu": "V100"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    if not args.no_match:
        # the metric's second half, on the same GPU after the timed region
        try:
            out["sound_match"] = sound_match(targets=args.match_targets,
                                             train_steps=args.match_train_steps,
                                             log=lambda *a: print(*a, file=sys.stderr, flush=True))
        except Exception as e:                      # the render line is still reported
            out["sound_match"] = {"error": f"{type(e).__name__}: {e}"}
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
