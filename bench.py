#!/usr/bin/env python3
"""Throughput of batched voice rendering on one MI355X.

Workload: 16384 voices of the default Voice, render lengths 1, 2 and 4 s
(by voice index mod 3) at 44.1 kHz packed back to back (1.686e9 samples,
6.74 GB of float32 audio), note durations uniform in [0.1, 4] s.  A step is
one pass of the hot path over the batch: the parameter draw (Philox) and the
fused render, with every input resident in HBM before the timed region.

Prints one JSON line: rendered samples/s (and MHz, x real time), the render
kernel's HBM roofline fraction measured with HIP events on its stream, and the
float64 CPU oracle timed on a bounded sample of the same workload.
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
RENDER_TRAFFIC = {"sources_sha256_16": "45cd108222b69c06",
                  "fetch_bytes": 10745190, "write_bytes": 6759242650, "valu_busy": 0.89}
RENDER_SOURCES = ("render.hip", "voice_device.h", "philox.h")


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
    ap.add_argument("--autotune", type=int, default=1,
                    help="time the candidate launch plans on this batch first (untimed) and "
                         "render with the fastest")
    ap.add_argument("--workload", default="render", choices=("render", "plain", "learned", "grad"),
                    help="render: the headline ragged render; plain: 128 voices x 4 s "
                         "(200 renders per timed step, in a HIP graph); learned: one proposal "
                         "training step (render + log-mel + MLP); grad: render, MR-STFT "
                         "loss and gradient, render adjoint")
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
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "launches": 3}), flush=True)


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
        S.synth_render(u, tab, n_samples=N, noise_seed=wl.key_noise(), out=out)
        torch.cuda.synchronize()
        g = torch.cuda.CUDAGraph()
        with torch.cuda.graph(g, stream=stream):
            for _ in range(reps):
                S.synth_render(u, tab, n_samples=N, noise_seed=wl.key_noise(), out=out)
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
                      "renders_per_step": reps},
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
    import torch
    import workloads as W
    import paper_2104_12922_amd as S

    wl = W.ragged_batch(args.batch)
    table = wl.nebula.table()
    dev = torch.device("cuda:0")
    torch.cuda.set_device(dev)
    B = wl.batch
    total = wl.total_samples
    offsets = torch.from_numpy(wl.offsets).to(dev)
    params = torch.empty(B, 78, dtype=torch.float32, device=dev)
    audio = torch.empty(total, dtype=torch.float32, device=dev)
    stream = torch.cuda.Stream(device=dev)

    # launch order: longest voices first (the lengths are known with the
    # offsets), so that short voices fill the end of the launch
    order = torch.from_numpy(np.argsort(-wl.lengths, kind="stable").astype(np.int32)).to(dev)
    lmax = int(wl.lengths.max())
    plan = (4, 1, 0, 0)                       # the library's default plan
    if args.rps:
        plan = (args.rps, 1, 0, 0)
    elif args.autotune:
        from paper_2104_12922_amd.autotune import RenderTuner
        with torch.cuda.stream(stream):
            S.synth_sample_params(wl.seed, wl.first_g, B, out=params)
            plan, _ = RenderTuner().tune(params, table, offsets=offsets, order=order,
                                         max_samples=lmax, noise_seed=wl.key_noise(), out=audio)
        torch.cuda.synchronize()

    def render():
        S.synth_render_plan(params, table, plan[0], plan[1], persistent=bool(plan[2]),
                            grid_blocks=plan[3], offsets=offsets,
                            carries=len(plan) > 4 and bool(plan[4]), max_samples=lmax,
                            order=order, noise_seed=wl.key_noise(), out=audio)

    def step():
        S.synth_sample_params(wl.seed, wl.first_g, B, out=params)
        render()

    with torch.cuda.stream(stream):
        step()
        torch.cuda.synchronize()
        # render-kernel time with HIP events on the stream the kernel runs on
        ev = [(torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True))
              for _ in range(max(3, min(args.steps, 10)))]
        for a, b in ev:
            a.record(stream)
            render()
            b.record(stream)
        torch.cuda.synchronize()
        kern_ms = float(np.mean([a.elapsed_time(b) for a, b in ev]))

        graph = None
        if args.graph:
            graph = torch.cuda.CUDAGraph()
            with torch.cuda.graph(graph, stream=stream):
                step()
            torch.cuda.synchronize()
        run = graph.replay if graph is not None else step

        for _ in range(args.warmup):
            run()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(args.steps):
            run()
        torch.cuda.synchronize()
        dt = time.perf_counter() - t0

    prof = render_traffic() if wl.batch == 16384 and plan in (None, (4, 1, 0, 0)) else None
    ms = dt / args.steps * 1e3
    value = total / (dt / args.steps)
    alg_bytes = 4.0 * total + 4.0 * 78 * B + 8.0 * (B + 1) + 4.0 * B   # audio, params, offsets, order
    achieved = alg_bytes / (kern_ms * 1e-3) / 1e9
    alu_tops = RENDER_SLOTS_PER_SAMPLE * total / (kern_ms * 1e-3) / 1e12
    out = {
        "metric": "rendered audio samples/sec", "value": value, "unit": "samples/s",
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
        # the render is bound by VALU issue: the roofline is the ALU one
        # (algorithmic slots / kernel time), with the HBM figures beside it
        "roofline": {"bound": "alu", "achieved": alu_tops, "peak": VALU_PEAK_TOPS,
                     "unit": "T VALU lane-slots/s", "frac": alu_tops / VALU_PEAK_TOPS,
                     "traffic": (float(prof["fetch_bytes"] + prof["write_bytes"])
                                 if prof else None),
                     "traffic_unit": "B/launch",
                     "slots_per_sample": RENDER_SLOTS_PER_SAMPLE,
                     "valu_busy_profiled": prof["valu_busy"] if prof else None,
                     "hbm": {"achieved": achieved, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                             "frac": achieved / HBM_PEAK_GBS, "alg_bytes_per_launch": alg_bytes},
                     "kernel": "render_kernel", "kernel_ms": kern_ms},
        "context": {"paper_single_gpu_mhz": 714.0, "paper_gpu": "V100"},
    }
    if not args.no_cpu_baseline:
        out["cpu_baseline"] = cpu_baseline(wl, args.cpu_seconds)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
