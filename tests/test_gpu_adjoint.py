"""GPU parity of the hand-written render adjoint (synth_render_backward)
against the float64 oracle's exact gradient (torch autograd), through the C ABI.

Criterion per voice (R25 form): |g_gpu - g_ref| <= tol * max(|g_ref|,
1e-3 * max|g_ref|) for every parameter, tol = 1e-3.  The adjoint's forward
recompute follows the render's float64 phase recurrences; the square-saw's
phase adjoint, a sum of large terms of both signs whose total can be 1e6
times smaller than their magnitudes for pitch parameters, is evaluated in
float64; the remaining float32 terms (sine VCO, amplitude-side sums) reach
about 1e-4.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox, spectral as sp, voice

pytestmark = pytest.mark.gpu
TOL = 1e-3


@pytest.fixture(scope="module")
def synth():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2104_12922_amd as S
    return S


def r25(g, ref):
    den = np.maximum(np.abs(ref), 1e-3 * np.abs(ref).max())
    return np.abs(g - ref) / den


def oracle_grad(u, g, N, table, noise_seed=0, first_g=0):
    x = torch.tensor(u, requires_grad=True)
    ids = np.arange(first_g, first_g + len(u))
    y = voice.render_uniform(x, ids, N, table, noise_seed=noise_seed)
    (y * torch.as_tensor(g, dtype=torch.float64)).sum().backward()
    return x.grad.numpy()


def check(ga, ref, tol=TOL):
    for b in range(len(ref)):
        rel = r25(ga[b], ref[b])
        worst = np.argsort(-rel)[:4]
        print("voice", b, "max rel %.3e" % rel.max(),
              [(int(p), "%.2e" % rel[p], "%.4e" % ref[b, p], "%.4e" % ga[b, p]) for p in worst],
              file=sys.stderr, flush=True)
        assert rel.max() <= tol, (b, rel.max(), int(rel.argmax()))


@pytest.mark.parametrize("N", [22050, 44100 + 37])
def test_adjoint_matches_oracle_random_cotangent(synth, N, nebula_table):
    B = 6
    u = philox.sample_params(3, np.arange(B)).astype(np.float32).astype(np.float64)
    g = np.random.default_rng(1).standard_normal((B, N)).astype(np.float32)
    ref = oracle_grad(u, g.astype(np.float64), N, nebula_table, noise_seed=2)
    ga = synth.synth_render_backward(torch.tensor(u, dtype=torch.float32).cuda(),
                                     torch.tensor(g).cuda(), nebula_table, noise_seed=2)
    torch.cuda.synchronize()
    check(ga.cpu().numpy().astype(np.float64), ref)


def test_adjoint_4s_and_curved_nebula(synth):
    tab = W.curved_test_nebula().table()
    B, N = 2, 176400
    u = philox.sample_params(7, np.arange(B)).astype(np.float32).astype(np.float64)
    g = np.random.default_rng(2).standard_normal((B, N)).astype(np.float32)
    ref = oracle_grad(u, g.astype(np.float64), N, tab, noise_seed=3, first_g=100)
    ga = synth.synth_render_backward(torch.tensor(u, dtype=torch.float32).cuda(),
                                     torch.tensor(g).cuda(), tab, noise_seed=3, first_g=100)
    torch.cuda.synchronize()
    check(ga.cpu().numpy().astype(np.float64), ref)


def test_loss_gradient_end_to_end(synth, nebula_table):
    """d MR-STFT(render(u), target) / du: GPU loss kernel + GPU adjoint vs the
    oracle's autograd through its own loss (float32 FFT tolerance)."""
    B, N = 4, 44100
    u = philox.sample_params(0, np.arange(B)).astype(np.float32).astype(np.float64)
    ut = philox.sample_params(1, np.arange(B))
    target = voice.render_uniform(torch.tensor(ut), np.arange(B), N, nebula_table, noise_seed=9)
    x = torch.tensor(u, requires_grad=True)
    sp.mrstft_loss_per_voice(voice.render_uniform(x, np.arange(B), N, nebula_table, noise_seed=0),
                             target).sum().backward()
    ref = x.grad.numpy()
    p = torch.tensor(u, dtype=torch.float32).cuda().requires_grad_(True)
    y = synth.SynthRender.apply(p, nebula_table, N, 0, 0)
    loss = synth.MRSTFTLoss.apply(y, target.float().cuda())
    loss.sum().backward()
    torch.cuda.synchronize()
    check(p.grad.cpu().numpy().astype(np.float64), ref, tol=3e-2)


def test_adjoint_deterministic_and_batch_independent(synth, nebula_table):
    B, N = 8, 30000
    u = torch.from_numpy(philox.sample_params(4, np.arange(B)).astype(np.float32)).cuda()
    g = torch.randn(B, N, device="cuda")
    a = synth.synth_render_backward(u, g, nebula_table, noise_seed=1)
    b = synth.synth_render_backward(u, g, nebula_table, noise_seed=1)
    c = synth.synth_render_backward(u[2:5].contiguous(), g[2:5].contiguous(), nebula_table,
                                    first_g=2, noise_seed=1)
    assert torch.equal(a, b)
    assert torch.equal(a[2:5], c)


def test_adjoint_argument_errors(synth, nebula_table):
    import ctypes
    from paper_2104_12922_amd import _native
    L = _native.lib()
    cfg, keep = _native.make_config(nebula_table, mix_mode=1)
    u = torch.rand(2, 78, device="cuda")
    g = torch.zeros(2, 1000, device="cuda")
    gp = torch.empty(2, 78, device="cuda")
    ws = torch.empty(1 << 20, dtype=torch.uint8, device="cuda")
    st = L.synth_render_backward(ctypes.byref(cfg), u.data_ptr(), None, 0, 2, 1000, g.data_ptr(),
                                 gp.data_ptr(), ws.data_ptr(), ws.numel(), None)
    assert st == -4                                       # mix mode 1 has no adjoint
    cfg0, keep0 = _native.make_config(nebula_table)
    st = L.synth_render_backward(ctypes.byref(cfg0), u.data_ptr(), None, 0, 2, 1000, g.data_ptr(),
                                 gp.data_ptr(), ws.data_ptr(), 10, None)
    assert st == -2                                       # workspace too small
    need = L.synth_render_backward_workspace(ctypes.byref(cfg0), 2, 1000)
    assert need == 2 * (10 * 21 + 1 * 88) * 8          # segment sums + one chunk's carries and totals


def test_adjoint_gradient_workload_all_256_voices(synth):
    """Gradient workload at full size: 256 voices x 4 s from seed 0, cotangent =
    the GPU MR-STFT gradient against targets of seed 1; the batched GPU adjoint
    against the oracle's autograd with the same cotangent, every voice."""
    wl = W.gradient_batch()
    tab = wl.nebula.table()
    N = 176400
    u = synth.synth_sample_params(wl.seed, 0, wl.batch)
    ut = synth.synth_sample_params(W.SEED_TARGET, 0, wl.batch)
    t = synth.synth_render(ut, tab, n_samples=N, noise_seed=W.SEED_TARGET)
    y = synth.synth_render(u, tab, n_samples=N, noise_seed=wl.seed)
    g_audio = synth.synth_mrstft_loss(y, t, grad=True)[1]
    ga = synth.synth_render_backward(u, g_audio, tab, noise_seed=wl.seed)
    torch.cuda.synchronize()
    ga = ga.cpu().numpy().astype(np.float64)
    uu = u.cpu().numpy().astype(np.float64)
    gc = g_audio.cpu().numpy().astype(np.float64)
    ref = np.concatenate([oracle_grad(uu[i:i + 32], gc[i:i + 32], N, tab, noise_seed=wl.seed,
                                      first_g=i) for i in range(0, wl.batch, 32)])
    check(ga, ref)


