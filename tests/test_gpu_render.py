"""GPU parity of the HIP render path against the float64 oracle, through the C ABI.

Bars: the parameter draw is bit-exact; audio samples (float32) are within
1e-4 max-abs of the float64 oracle render.
"""
import math
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox, voice

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def synth():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2104_12922_amd as S
    return S


def say(*a):
    print(*a, file=sys.stderr, flush=True)


def oracle_render(u, ids, lengths, table, sr=44100.0, rc=441.0, noise_seed=0, mix_mode=0):
    return voice.render(torch.as_tensor(u, dtype=torch.float64), ids, lengths, table, sr, rc,
                        noise_seed, mix_mode).numpy()


# ---------------------------------------------------------------------------
# parameter draw
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed,first_g,B", [(0, 0, 128), (1, 5, 37), (2**63 + 12345, 2**33 - 3, 300)])
def test_sample_params_bit_exact(synth, seed, first_g, B):
    say("sample_params", seed, first_g, B)
    got = synth.synth_sample_params(seed, first_g, B).cpu().numpy()
    exp = philox.sample_params(seed, np.arange(B, dtype=np.uint64) + np.uint64(first_g))
    assert got.dtype == np.float32
    assert np.array_equal(got.astype(np.float64), exp)


def test_sample_params_voice_ids(synth):
    ids = np.array([7, 2**40 + 1, 3, 2**64 - 1], dtype=np.uint64)
    got = synth.synth_sample_params(9, voice_ids=torch.from_numpy(ids.view(np.int64)).cuda())
    assert np.array_equal(got.cpu().numpy().astype(np.float64), philox.sample_params(9, ids))


# ---------------------------------------------------------------------------
# render parity
# ---------------------------------------------------------------------------
def gpu_render(synth, u, table, lengths=None, n=None, ids=None, first_g=0, **kw):
    p = torch.as_tensor(np.asarray(u, dtype=np.float32)).cuda()
    if lengths is not None:
        off = np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)
        y = synth.synth_render(p, table, offsets=torch.from_numpy(off).cuda(),
                               voice_ids=None if ids is None else
                               torch.from_numpy(np.asarray(ids, np.uint64).view(np.int64)).cuda(),
                               first_g=first_g, **kw)
    else:
        y = synth.synth_render(p, table, n_samples=n, first_g=first_g, **kw)
    torch.cuda.synchronize()
    return y.cpu().numpy().astype(np.float64)


def test_plain_render_b128_4s_matches_oracle(synth):
    """The plain render: 128 voices x 4 s at 44.1 kHz, every sample compared."""
    wl = W.plain_render()
    say("plain render", wl.name)
    table = wl.nebula.table()
    u = synth.synth_sample_params(wl.seed, 0, wl.batch)
    y = synth.synth_render(u, table, n_samples=176400, noise_seed=wl.key_noise())
    torch.cuda.synchronize()
    got = y.cpu().numpy().astype(np.float64)
    ref = voice.render_uniform(torch.from_numpy(u.cpu().numpy().astype(np.float64)),
                               np.arange(wl.batch), 176400, table, noise_seed=wl.key_noise()).numpy()
    err = np.abs(got - ref)
    say("max abs err", err.max(), "at", np.unravel_index(err.argmax(), err.shape))
    assert np.isfinite(got).all()
    assert err.max() <= TOL
    # the exactly silent tail is exactly zero
    js = voice.silence_start(u.cpu().numpy().astype(np.float64), table)
    for b in range(wl.batch):
        s = (int(math.floor(js[b])) + 2) * 100
        if s < 176400:
            assert (got[b, s:] == 0).all()


@pytest.mark.parametrize("lengths", [
    [1, 7, 8, 9, 99, 100, 101, 6199, 6200, 6201, 12400, 3333],
    [44100, 88200, 176400],
])
def test_ragged_lengths_match_oracle(synth, lengths, nebula_table):
    say("ragged", lengths)
    B = len(lengths)
    u = philox.sample_params(5, np.arange(B))
    got = gpu_render(synth, u, nebula_table, lengths=np.array(lengths), noise_seed=77)
    ref = oracle_render(u, np.arange(B), lengths, nebula_table, noise_seed=77)
    assert got.shape == ref.shape
    assert np.abs(got - ref).max() <= TOL


def test_voice_ids_and_first_g(synth, nebula_table):
    ids = np.array([2**33 + 17, 5, 123456789], dtype=np.uint64)
    u = philox.sample_params(3, ids)
    got = gpu_render(synth, u, nebula_table, lengths=np.array([5000, 5000, 5000]), ids=ids, noise_seed=4)
    ref = oracle_render(u, ids, [5000] * 3, nebula_table, noise_seed=4)
    assert np.abs(got - ref).max() <= TOL
    got2 = gpu_render(synth, u, nebula_table, n=5000, first_g=1000, noise_seed=4).reshape(-1)
    ref2 = oracle_render(u, np.arange(1000, 1003), [5000] * 3, nebula_table, noise_seed=4)
    assert np.abs(got2 - ref2).max() <= TOL


@pytest.mark.parametrize("sr,rc", [(28224.0, 441.0), (88200.0, 441.0), (8000.0, 80.0), (4410.0, 44.1)])
def test_other_rates_and_nyquist_clamp(synth, sr, rc, nebula_table):
    """q = 64 and 200, a rate where high pitches exceed sr/2 (clamped path), q = 100 at 4.41 kHz."""
    say("rates", sr, rc)
    u = philox.sample_params(8, np.arange(16))
    n = int(2.5 * sr)
    got = gpu_render(synth, u, nebula_table, n=n, sample_rate=sr, control_rate=rc, noise_seed=1)
    ref = voice.render_uniform(torch.tensor(u), np.arange(16), n, nebula_table, sr, rc, 1).numpy()
    assert np.abs(got.reshape(16, n) - ref).max() <= TOL


def test_curved_nebula_and_mix_mode_1(synth):
    tab = W.curved_test_nebula().table()
    u = philox.sample_params(21, np.arange(24))
    u[:, 75:78] = np.maximum(u[:, 75:78], 0.9)
    for mode in (0, 1):
        got = gpu_render(synth, u, tab, n=30000, noise_seed=2, mix_mode=mode)
        ref = voice.render_uniform(torch.tensor(u), np.arange(24), 30000, tab, noise_seed=2,
                                   mix_mode=mode).numpy()
        assert np.abs(got.reshape(24, -1) - ref).max() <= TOL
        if mode == 1:
            assert np.abs(got).max() <= 1.0 + 1e-6


def test_launch_plans_bit_identical(synth, nebula_table):
    """Slicing a voice over workgroups and persistent scheduling change nothing."""
    u = torch.from_numpy(philox.sample_params(0, np.arange(40)).astype(np.float32)).cuda()
    base = synth.synth_render_plan(u, nebula_table, 4, 1, n_samples=176400)
    for rps, slices, pers, grid in [(4, 3, False, 0), (4, 7, False, 0), (4, 1, True, 13),
                                    (4, 2, True, 5)]:
        y = synth.synth_render_plan(u, nebula_table, rps, slices, pers, grid, n_samples=176400)
        assert torch.equal(y, base), (rps, slices, pers, grid)
    ref = voice.render_uniform(torch.from_numpy(u.cpu().numpy().astype(np.float64)), np.arange(40),
                               176400, nebula_table).numpy()
    for rps in (1, 2):
        y = synth.synth_render_plan(u, nebula_table, rps, 1, n_samples=176400)
        torch.cuda.synchronize()
        assert np.abs(y.cpu().numpy() - ref).max() <= TOL, rps


def test_ragged_slices_bit_identical(synth):
    """Splitting ragged voices over workgroups (including voices shorter than
    the number of slices' worth of chunks, and empty voices) changes nothing."""
    lengths = np.array([44100, 0, 1, 6200, 176400, 99, 88200, 132300, 12401, 176400])
    off = torch.from_numpy(np.concatenate([[0], np.cumsum(lengths)]).astype(np.int64)).cuda()
    tab = W.default_nebula(duration_min=0.1).table()
    u = synth.synth_sample_params(4, 0, lengths.size)
    base = synth.synth_render_plan(u, tab, 4, 1, offsets=off, noise_seed=4)
    for sl in (2, 3, 8):
        for car in (False, True):
            y = synth.synth_render_plan(u, tab, 4, sl, offsets=off, noise_seed=4, carries=car)
            assert torch.equal(y, base), (sl, car)
    y = synth.synth_render_plan(u, tab, 4, 4, True, 7, offsets=off, noise_seed=4)
    assert torch.equal(y, base)
    # carries sized for 1 s: longer voices' later slices walk their chunks
    y = synth.synth_render_plan(u, tab, 4, 8, offsets=off, noise_seed=4, max_samples=44100)
    assert torch.equal(y, base)
    # the order in which workgroups take the voices changes nothing
    for perm in (np.argsort(-lengths, kind="stable"), np.random.default_rng(3).permutation(lengths.size)):
        order = torch.from_numpy(perm.astype(np.int32)).cuda()
        for sl, pers in ((1, False), (3, False), (2, True)):
            y = synth.synth_render_plan(u, tab, 4, sl, pers, 3 if pers else 0, offsets=off,
                                        noise_seed=4, order=order)
            assert torch.equal(y, base), (sl, pers)


def test_autotuner_picks_a_plan_and_renders_with_it(synth):
    from paper_2104_12922_amd.autotune import RenderTuner
    wl = W.ragged_batch(600)
    tab = wl.nebula.table()
    offs = torch.from_numpy(wl.offsets).cuda()
    u = synth.synth_sample_params(wl.seed, 0, wl.batch)
    tuner = RenderTuner(reps=1)
    plan, times = tuner.tune(u, tab, offsets=offs, noise_seed=wl.key_noise())
    assert plan in times and len(times) >= 2
    y = tuner.render(u, tab, offsets=offs, noise_seed=wl.key_noise())
    z = synth.synth_render_plan(u, tab, plan[0], plan[1], bool(plan[2]), plan[3], offsets=offs,
                                carries=len(plan) > 4 and bool(plan[4]),
                                noise_seed=wl.key_noise())
    d = synth.synth_render(u, tab, offsets=offs, noise_seed=wl.key_noise())
    assert torch.equal(y, z)
    assert float((y - d).abs().max()) <= 1e-5


def test_batch_independence_and_determinism(synth, nebula_table):
    u = synth.synth_sample_params(0, 0, 64)
    a = synth.synth_render(u, nebula_table, n_samples=50000)
    b = synth.synth_render(u, nebula_table, n_samples=50000)
    c = synth.synth_render(u[10:20].contiguous(), nebula_table, n_samples=50000, first_g=10)
    assert torch.equal(a, b)
    assert torch.equal(a[10:20], c)


def test_empty_batch_is_noop(synth, nebula_table):
    u = torch.empty(0, 78, device="cuda")
    y = synth.synth_render(u, nebula_table, n_samples=100)
    assert y.numel() == 0


def test_ragged_batch_b16384_sampled_against_oracle(synth):
    """Batched-throughput workload at full size: 16384 voices of 1, 2 and 4 s,
    packed; 36 voices compared with the oracle, properties checked on all."""
    wl = W.ragged_batch()
    table = wl.nebula.table()
    say("ragged full", wl.name, wl.total_samples)
    u = synth.synth_sample_params(wl.seed, 0, wl.batch)
    off = torch.from_numpy(wl.offsets).cuda()
    y = synth.synth_render(u, table, offsets=off, noise_seed=wl.key_noise())
    torch.cuda.synchronize()
    assert y.numel() == wl.total_samples
    assert bool(torch.isfinite(y).all())
    assert float(y.abs().max()) <= 3.125
    pick = np.concatenate([np.arange(0, 12), np.arange(8190, 8202), np.arange(16372, 16384)])
    uu = u[torch.from_numpy(pick).cuda()].cpu().numpy().astype(np.float64)
    ref = oracle_render(uu, pick, wl.lengths[pick], table, noise_seed=wl.key_noise())
    offs = wl.offsets
    got = np.concatenate([y[offs[i]:offs[i + 1]].cpu().numpy() for i in pick]).astype(np.float64)
    assert np.abs(got - ref).max() <= TOL


def test_timed_bench_step_matches_oracle(synth):
    """The exact step the throughput benchmark times (bench.RenderStep: the
    parameter draw and the ragged 16384-voice render with the autotuned launch
    plan and the longest-first voice order, captured in HIP graphs), after
    three graph replays: the parameters of every voice bit-exact, 256 sampled
    voices (a third of each length, 1, 2 and 4 s) against the oracle."""
    import bench
    wl = W.ragged_batch()
    st = bench.RenderStep(wl)
    say("bench step plan", st.plan)
    for _ in range(3):
        st.run()
    torch.cuda.synchronize()
    assert st.graphs is not None
    u = st.params.cpu().numpy().astype(np.float64)
    assert np.array_equal(u, philox.sample_params(wl.seed, np.arange(wl.batch, dtype=np.uint64)))
    rng = np.random.default_rng(7)
    pick = np.sort(np.concatenate([rng.choice(np.nonzero(wl.lengths == n)[0], 86 if k < 2 else 84,
                                              replace=False)
                                   for k, n in enumerate(np.unique(wl.lengths))]))
    assert len(pick) == 256
    y = st.audio
    assert bool(torch.isfinite(y).all())
    ref = oracle_render(u[pick], pick, wl.lengths[pick], st.table, noise_seed=wl.key_noise())
    offs = wl.offsets
    got = np.concatenate([y[offs[i]:offs[i + 1]].cpu().numpy() for i in pick]).astype(np.float64)
    err = np.abs(got - ref).max()
    say("bench step: 256 sampled voices, max |gpu - oracle| = %.3e" % err)
    assert err <= TOL


def test_malformed_offsets_stay_inside_the_buffer(synth, nebula_table):
    """Offsets that decrease ([0, 100, 50, 60]) are a caller error; the
    kernels cut every voice's range to [0, offsets[batch]), so nothing is
    written outside the 60-sample buffer (a guard region after it stays
    untouched) and the voices that fit are rendered as for valid offsets."""
    u = synth.synth_sample_params(3, 0, 3)
    buf = torch.full((60 + 4096,), 7.0, device="cuda")
    offs = torch.tensor([0, 100, 50, 60], dtype=torch.int64, device="cuda")
    synth.synth_render(u, nebula_table, offsets=offs, out=buf[:60])
    torch.cuda.synchronize()
    assert bool((buf[60:] == 7.0).all())
    ok = synth.synth_render(u, nebula_table, n_samples=60)
    torch.cuda.synchronize()
    assert torch.equal(buf[:50], ok[0, :50])            # voice 0, cut to the buffer
    # [50, 60) is written by voice 0 (cut) and voice 2: either value
    tail = buf[50:60]
    assert bool(((tail == ok[0, 50:60]) | (tail == ok[2, :10])).all())
