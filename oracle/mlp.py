"""Reference of the learned proposal's arithmetic (float64 on the CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

MLP d_in -> d_h -> d_h -> d_out with erf-GELU hidden units and a sigmoid
output, trained on the mean squared error to the normalised parameters.  With
round_bf16=True the operands are rounded to bfloat16 at the points where the
GPU path stores bf16 (input, weights, h1, h2, and the backward's dz3, dh2,
dh1), so that both sides take the same quantisation decisions; accumulation
is float64 here and float32 on the GPU.  With round_bf16=False the manual
backward is the plain chain rule and is pinned against torch autograd; that
plain form, given only bf16-rounded inputs and weights, is what the GPU path
is held to (the rounding-point variant is a secondary diagnostic).

adam_step is Adam (Kingma and Ba, ICLR 2015, Algorithm 1) with bias
correction, written from that algorithm and pinned against torch.optim.Adam.
"""
from __future__ import annotations

import math

import torch

F64 = torch.float64


def bf16(x: torch.Tensor) -> torch.Tensor:
    """Round to the nearest bfloat16 (ties to even) through float32."""
    return x.float().to(torch.bfloat16).to(F64)


def gelu(x):
    return 0.5 * x * (1.0 + torch.erf(x / math.sqrt(2.0)))


def gelu_grad(x):
    return 0.5 * (1.0 + torch.erf(x / math.sqrt(2.0))) + x * torch.exp(-0.5 * x * x) / math.sqrt(2.0 * math.pi)


def forward(x, w, round_bf16=True):
    """x [B, d_in]; w dict of w1t [d_h, d_in], b1, w2t, b2, w3t, b3.  Returns dict."""
    r = bf16 if round_bf16 else (lambda t: t.to(F64))
    x = r(torch.as_tensor(x))
    W1, W2, W3 = (r(torch.as_tensor(w[k])) for k in ("w1t", "w2t", "w3t"))
    b1, b2, b3 = (torch.as_tensor(w[k]).to(F64) for k in ("b1", "b2", "b3"))
    h1pre = x @ W1.T + b1
    h1 = r(gelu(h1pre))
    h2pre = h1 @ W2.T + b2
    h2 = r(gelu(h2pre))
    out = torch.sigmoid(h2 @ W3.T + b3)
    return {"x": x, "h1pre": h1pre, "h1": h1, "h2pre": h2pre, "h2": h2, "out": out,
            "W2": W2, "W3": W3}


def backward(f, target, round_bf16=True):
    """Gradients of mean((out - target)^2) (chain rule written out)."""
    r = bf16 if round_bf16 else (lambda t: t)
    out = f["out"]
    B, D = out.shape
    t = torch.as_tensor(target).to(F64)
    loss = ((out - t) ** 2).mean()
    dz3 = r(2.0 * (out - t) / (B * D) * out * (1.0 - out))
    g = {"w3t": dz3.T @ f["h2"], "b3": dz3.sum(0)}
    dh2 = r((dz3 @ f["W3"]) * gelu_grad(f["h2pre"]))
    g["w2t"] = dh2.T @ f["h1"]
    g["b2"] = dh2.sum(0)
    dh1 = r((dh2 @ f["W2"]) * gelu_grad(f["h1pre"]))
    g["w1t"] = dh1.T @ f["x"]
    g["b1"] = dh1.sum(0)
    return loss, g


def adam_step(w, g, m, v, t, lr, beta1=0.9, beta2=0.999, eps=1e-8):
    """One Adam update at step t >= 1 (Kingma and Ba, Algorithm 1): the moment
    estimates m, v are updated from the gradient g, bias-corrected by
    1 - beta^t, and w moves by lr m_hat / (sqrt(v_hat) + eps).  Float64;
    returns (w, m, v)."""
    w, g, m, v = (torch.as_tensor(a).to(F64) for a in (w, g, m, v))
    m = beta1 * m + (1.0 - beta1) * g
    v = beta2 * v + (1.0 - beta2) * g * g
    m_hat = m / (1.0 - beta1 ** t)
    v_hat = v / (1.0 - beta2 ** t)
    return w - lr * m_hat / (torch.sqrt(v_hat) + eps), m, v
