"""GPU parity of the multi-resolution STFT loss and its gradient against the
float64 oracle (autograd of the oracle loss), through the C ABI.

Tolerances come from the arithmetic.  The loss is a mean of float32 log
differences accumulated in float64: 1e-5 relative.  The gradient is compared
element by element, per voice, relative to the voice's largest gradient
magnitude: e = max_n |g(n) - g_ref(n)| / max_n |g_ref(n)|.  The float32
floor of that measure is what the same definition evaluated with float32
FFTs and float32 autograd on the CPU (``loss32``) reaches, e32; both
evaluations round the frame, the transform, |X| and the log in float32, and
the GPU's transform and hardware log2 / sqrt / reciprocal add a few ulp per
step, so the GPU is held to e <= 16 e32 for every voice (no absolute floor).
A voice with an exactly zero reference gradient must get exactly zero.
"""
import sys

import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox, spectral as sp, voice

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def synth():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2104_12922_amd as S
    return S


def renders(seed, B, N):
    u = philox.sample_params(seed, np.arange(B))
    return voice.render_uniform(torch.tensor(u), np.arange(B), N, W.default_nebula().table(),
                                noise_seed=seed).float()


def loss32(x, t):
    """The same definition evaluated with float32 FFTs on the CPU."""
    tot = torch.zeros(x.shape[0])
    for n in sp.MR_SIZES:
        if sp.num_frames(x.shape[-1], n, n // 4) == 0:
            continue
        w = sp.hann(n).float()
        X = torch.fft.rfft(sp.frames(x, n, n // 4) * w, dim=-1).abs()
        T = torch.fft.rfft(sp.frames(t, n, n // 4) * w, dim=-1).abs()
        tot = tot + (torch.log(X + 1e-5) - torch.log(T + 1e-5)).abs().mean(dim=(-2, -1))
    return tot


GRAD_FACTOR = 16.0


def check(synth, x32, t32, loss_rtol=1e-5, factor=GRAD_FACTOR):
    x64, t64 = x32.double(), t32.double()
    xr = x64.clone().requires_grad_(True)
    ref = sp.mrstft_loss_per_voice(xr, t64)
    ref.sum().backward()
    xf = x32.clone().requires_grad_(True)
    loss32(xf, t32).sum().backward()
    loss, g = synth.synth_mrstft_loss(x32.cuda(), t32.cuda(), grad=True)
    torch.cuda.synchronize()
    loss, g = loss.cpu(), g.cpu().double()
    print("loss", loss.numpy()[:4], "ref", ref.detach().numpy()[:4], file=sys.stderr, flush=True)
    assert torch.allclose(loss, ref.detach(), rtol=loss_rtol, atol=1e-9)
    for b in range(x32.shape[0]):
        gr = xr.grad[b]
        gmax = float(gr.abs().max())
        if gmax == 0:
            assert float(g[b].abs().max()) == 0.0
            continue
        err = float((g[b] - gr).abs().max()) / gmax
        err32 = float((xf.grad[b].double() - gr).abs().max()) / gmax
        print("voice", b, "grad max-abs rel %.3e" % err, "cpu float32 %.3e" % err32,
              "ratio %.2f" % (err / err32 if err32 > 0 else float("inf")), file=sys.stderr, flush=True)
        assert err <= factor * err32, (b, err, err32)


def test_mrstft_loss_and_grad_4s(synth):
    x = renders(0, 6, 176400)
    t = renders(1, 6, 176400)
    check(synth, x, t)


@pytest.mark.parametrize("N", [600, 1500, 2048, 5000, 44100])
def test_mrstft_short_and_ragged_frame_counts(synth, N):
    x = renders(2, 3, N)
    t = renders(3, 3, N)
    check(synth, x, t)


def test_mrstft_degenerate_cases(synth):
    x = renders(4, 2, 8000)
    loss, g = synth.synth_mrstft_loss(x.cuda(), x.cuda(), grad=True)
    assert float(loss.abs().max()) == 0.0 and float(g.abs().max()) == 0.0
    short = torch.randn(2, 300)
    loss, g = synth.synth_mrstft_loss(short.cuda(), torch.zeros(2, 300).cuda(), grad=True)
    assert float(loss.abs().max()) == 0.0 and float(g.abs().max()) == 0.0   # no frame fits
    silent = torch.zeros(2, 4096)
    loss = synth.synth_mrstft_loss(silent.cuda(), silent.cuda())
    assert float(loss.abs().max()) == 0.0


def test_mrstft_deterministic_and_loss_only_matches(synth):
    x = renders(5, 4, 30000).cuda()
    t = renders(6, 4, 30000).cuda()
    l1, g1 = synth.synth_mrstft_loss(x, t, grad=True)
    l2, g2 = synth.synth_mrstft_loss(x, t, grad=True)
    l3 = synth.synth_mrstft_loss(x, t)
    assert torch.equal(l1, l2) and torch.equal(g1, g2) and torch.equal(l1, l3)


def test_mrstft_gradient_batch_b256_4s_sampled(synth):
    """Gradient workload size: 256 voices x 4 s against targets from another seed;
    4 voices compared with the oracle, every voice checked for finiteness."""
    wl = W.gradient_batch()
    tab = wl.nebula.table()
    u = synth.synth_sample_params(wl.seed, 0, wl.batch)
    ut = synth.synth_sample_params(W.SEED_TARGET, 0, wl.batch)
    x = synth.synth_render(u, tab, n_samples=176400, noise_seed=wl.seed)
    t = synth.synth_render(ut, tab, n_samples=176400, noise_seed=W.SEED_TARGET)
    loss, g = synth.synth_mrstft_loss(x, t, grad=True)
    torch.cuda.synchronize()
    assert bool(torch.isfinite(loss).all()) and bool(torch.isfinite(g).all())
    pick = list(range(0, 256, 17)) + [255]
    check(synth, x[pick].cpu(), t[pick].cpu())


def test_mrstft_gradient_of_tiny_bins(synth):
    """Bins far below float32's squared range (|X| around 1e-22, as in quiet
    release tails) keep their magnitude and their gradient, whose size
    1 / (|X| + 1e-5) is the largest any bin has."""
    g = torch.Generator().manual_seed(5)
    x = torch.randn(3, 6000, generator=g) * 0.3
    x[0] *= 1e-21                       # every bin tiny
    x[1, 3000:] *= 1e-24                # a tiny second half
    x[2, :2500] *= 1e-30                # tiny frames ahead of loud ones
    t = torch.randn(3, 6000, generator=g) * 0.3
    t[2] *= 1e-22                       # tiny target
    check(synth, x, t)


@pytest.mark.parametrize("B,N", [(3, 300), (3, 600), (5, 5000), (4, 44100), (256, 176400)])
def test_mrstft_cached_target_is_bitwise_uncached(synth, B, N):
    """Target spectra computed once (synth_mrstft_target) give bitwise the loss
    and gradient of the uncached call, for two different renders against the
    same cached target, with and without a gradient."""
    x = renders(7, B, N).cuda() if B <= 8 else torch.randn(B, N).cuda() * 0.3
    x2 = renders(8, B, N).cuda() if B <= 8 else torch.randn(B, N).cuda() * 0.3
    t = renders(9, B, N).cuda() if B <= 8 else torch.randn(B, N).cuda() * 0.3
    tc = synth.synth_mrstft_target(t)
    for xi in (x, x2):
        l0, g0 = synth.synth_mrstft_loss(xi, t, grad=True)
        l1, g1 = synth.synth_mrstft_loss(xi, tc, grad=True)
        l2 = synth.synth_mrstft_loss(xi, tc)
        torch.cuda.synchronize()
        assert torch.equal(l0, l1) and torch.equal(g0, g1) and torch.equal(l0, l2)
    lt = synth.synth_mrstft_loss(t, tc)
    assert float(lt.abs().max()) == 0.0
