"""Pins of the proposal-network reference: the written-out chain rule equals
torch autograd, GELU' is the derivative of GELU, bf16 rounding is
round-to-nearest-even, and the bf16 log-mel stays within bf16 error of the
float64 one."""
import math

import numpy as np
import torch

import workloads as W
from oracle import mlp, spectral as sp, voice, philox

F64 = torch.float64


def small_weights(seed=0, d_in=64, d_h=32, d_out=78):
    w = W.mlp_init(seed, d_in, d_h, d_out)
    rng = np.random.default_rng(seed + 1)
    w["b1"] = rng.standard_normal(d_h).astype(np.float32) * 0.1
    w["b2"] = rng.standard_normal(d_h).astype(np.float32) * 0.1
    w["b3"] = rng.standard_normal(d_out).astype(np.float32) * 0.1
    return w


def test_manual_backward_equals_autograd():
    w = small_weights()
    rng = np.random.default_rng(3)
    x = torch.tensor(rng.standard_normal((17, 64)))
    t = torch.tensor(rng.random((17, 78)))
    f = mlp.forward(x, w, round_bf16=False)
    loss, g = mlp.backward(f, t, round_bf16=False)
    wt = {k: torch.tensor(v, dtype=F64, requires_grad=True) for k, v in w.items()}
    h1 = mlp.gelu(x @ wt["w1t"].T + wt["b1"])
    h2 = mlp.gelu(h1 @ wt["w2t"].T + wt["b2"])
    out = torch.sigmoid(h2 @ wt["w3t"].T + wt["b3"])
    ref = ((out - t) ** 2).mean()
    ref.backward()
    assert abs(float(loss) - float(ref)) < 1e-14
    for k in wt:
        assert torch.allclose(g[k], wt[k].grad, rtol=1e-10, atol=1e-14), k


def test_gelu_grad_is_derivative():
    x = torch.linspace(-6, 6, 1001, dtype=F64, requires_grad=True)
    mlp.gelu(x).sum().backward()
    assert torch.allclose(mlp.gelu_grad(x.detach()), x.grad, atol=1e-14)
    assert float(mlp.gelu(torch.tensor(0.0, dtype=F64))) == 0.0
    assert abs(float(mlp.gelu(torch.tensor(10.0, dtype=F64))) - 10.0) < 1e-12


def test_bf16_rounding_is_nearest_even():
    v = torch.tensor([1.0, 1.0 + 2 ** -8, 1.0 + 3 * 2 ** -8, 1.0 + 2 ** -9, 1.0 + 3 * 2 ** -9], dtype=F64)
    r = mlp.bf16(v)
    assert r.tolist() == [1.0, 1.0, 1.0 + 2 ** -6, 1.0, 1.0 + 2 ** -7]


def test_logmel_bf16_within_bf16_error_of_float64():
    u = philox.sample_params(0, np.arange(2))
    x = voice.render_uniform(torch.tensor(u), np.arange(2), 176400, W.default_nebula().table())
    a = sp.logmel(x)
    b = sp.logmel_bf16(x)
    d = (a - b).abs()
    # bf16 frames and basis give ~2^-9 relative error per product; loud bands
    # move by ~1e-2 in log, bands at the float64 floor (log 1e-6) by more
    loud = a > math.log(1e-3)
    assert float(d[loud].median()) < 2e-2
    assert (b.argmax(1) == a.argmax(1)).float().mean() > 0.9


def test_logmel_p16_within_bf16_rounding_of_float64():
    """Rounding only the power spectrum and the mel basis to bf16 moves a loud
    band by at most the two roundings (2 x 2^-9 relative, ~4e-3 in log)."""
    u = philox.sample_params(1, np.arange(2))
    x = voice.render_uniform(torch.tensor(u), np.arange(2), 176400, W.default_nebula().table())
    a = sp.logmel(x)
    b = sp.logmel_p16(x)
    loud = a > math.log(1e-2)
    assert bool(loud.any())
    assert float((a - b).abs()[loud].max()) < 1e-2
    assert float((a - b).abs()[loud].median()) < 3e-3


def test_adam_step_matches_torch_optim_adam():
    """The oracle's Adam against the library routine (torch.optim.Adam, float64)
    over five steps with changing gradients."""
    g = torch.Generator().manual_seed(4)
    w0 = torch.randn(50, generator=g, dtype=F64)
    grads = [torch.randn(50, generator=g, dtype=F64) for _ in range(5)]
    p = torch.nn.Parameter(w0.clone())
    opt = torch.optim.Adam([p], lr=3e-3, betas=(0.9, 0.999), eps=1e-8)
    w, m, v = w0.clone(), torch.zeros(50, dtype=F64), torch.zeros(50, dtype=F64)
    for t, gk in enumerate(grads, start=1):
        p.grad = gk.clone()
        opt.step()
        w, m, v = mlp.adam_step(w, gk, m, v, t, 3e-3)
        assert torch.allclose(w, p.detach(), rtol=0, atol=1e-15), t
