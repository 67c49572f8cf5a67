"""Resonant low-pass filter and its adjoint on the GPU against the float64
oracle (oracle/filter.py), through the C ABI.

Bounds.  Forward: the kernel keeps state and coefficients in float64 and
rounds y to float32 once, so |y - y_ref| <= 2^-24 |y_ref| + 1e-9 max|y_ref|
(the second term covers float64 reordering in the chunk scan and the
coefficient functions, amplified by the resonance).  Adjoint: lambda is kept
in LDS as float32 between passes, so dL/dx is within 2^-22 of the scale of
its three terms, and the coefficient-gradient sums within 1e-5 relative."""
import numpy as np
import pytest
import torch

from oracle import filter as OF

pytestmark = pytest.mark.gpu

SR = 44100.0
U = 2.0 ** -24


@pytest.fixture(scope="module")
def V():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2104_12922_amd import vcf
    return vcf


def _inputs(B, N, seed, period=100):
    g = np.random.default_rng(seed)
    t = np.arange(N) / SR
    f0 = g.uniform(55, 880, size=(B, 1))
    saw = 2.0 * ((t[None, :] * f0) % 1.0) - 1.0
    x = (0.6 * saw + 0.2 * g.standard_normal((B, N))).astype(np.float32)
    J = (N + period - 1) // period + 1
    env = np.clip(np.cumsum(g.uniform(-0.1, 0.12, size=(B, J)), axis=1), 0, 1).astype(np.float32)
    params = np.stack([g.uniform(30, 100, B), g.uniform(-24, 48, B), g.uniform(0.5, 15, B)],
                      axis=1).astype(np.float32)
    return x, env, params


def _ref(x, env, params, period=100):
    p = params.astype(np.float64)
    return OF.lowpass(x.astype(np.float64), env.astype(np.float64), p[:, 0], p[:, 1], p[:, 2],
                      period, SR).numpy()


def _check_y(y, ref):
    bound = U * np.abs(ref) + 1e-9 * max(1.0, np.max(np.abs(ref)))
    err = np.abs(y.astype(np.float64) - ref)
    assert np.all(err <= bound), (np.max(err / bound), np.argmax(err / bound))


@pytest.mark.parametrize("B,N,period", [(4, 12957, 100), (3, 6400, 100), (2, 6401, 100),
                                        (2, 700, 4), (2, 5000, 256), (5, 3, 100)])
def test_forward_matches_oracle(V, B, N, period):
    x, env, params = _inputs(B, N, N + B, period)
    y = V.lowpass(torch.from_numpy(x).cuda(), torch.from_numpy(env).cuda(),
                  torch.from_numpy(params).cuda(), period, SR).cpu().numpy()
    _check_y(y, _ref(x, env, params, period))


def test_ragged_voices_and_in_place(V):
    lens = [1, 2, 3, 99, 100, 101, 6400, 6401, 12802, 0, 250]
    B = len(lens)
    N = max(lens)
    x, env, params = _inputs(B, N, 7)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    packed = np.concatenate([x[b, :l] for b, l in enumerate(lens)])
    xp = torch.from_numpy(packed).cuda()
    y = V.lowpass(xp, torch.from_numpy(env).cuda(), torch.from_numpy(params).cuda(), 100, SR,
                  offsets=torch.from_numpy(offs).cuda(), max_samples=N).cpu().numpy()
    for b, l in enumerate(lens):
        if l == 0:
            continue
        ref = _ref(x[b:b + 1, :l], env[b:b + 1], params[b:b + 1])[0]
        _check_y(y[offs[b]:offs[b + 1]], ref)
    # in place: y over x
    xi = xp.clone()
    V.lowpass(xi, torch.from_numpy(env).cuda(), torch.from_numpy(params).cuda(), 100, SR,
              offsets=torch.from_numpy(offs).cuda(), max_samples=N, out=xi)
    assert np.array_equal(xi.cpu().numpy(), y)


def _oracle_grads(x, env, params, w, period=100):
    xt = torch.tensor(x.astype(np.float64), requires_grad=True)
    et = torch.tensor(env.astype(np.float64), requires_grad=True)
    pt = torch.tensor(params.astype(np.float64), requires_grad=True)
    y = OF.lowpass(xt, et, pt[:, 0], pt[:, 1], pt[:, 2], period, SR)
    (y * torch.tensor(w.astype(np.float64))).sum().backward()
    return xt.grad.numpy(), pt.grad.numpy(), et.grad.numpy()


@pytest.mark.parametrize("B,N,period", [(3, 2530, 100), (2, 6500, 100), (2, 400, 4), (2, 4161, 64),
                                        (2, 2600, 256), (2, 1500, 36)])
def test_backward_matches_oracle(V, B, N, period):
    x, env, params = _inputs(B, N, 100 + N, period)
    w = np.random.default_rng(N).standard_normal((B, N)).astype(np.float32)
    X, E, P = (torch.from_numpy(a).cuda() for a in (x, env, params))
    y, st = V.lowpass(X, E, P, period, SR, keep_states=True)
    gx, gp, ge = V.lowpass_backward(X, torch.from_numpy(w).cuda(), E, P, st, period, SR)
    rx, rp, re = _oracle_grads(x, env, params, w, period)
    gx, gp, ge = gx.cpu().numpy(), gp.cpu().numpy(), ge.cpu().numpy()
    scale = np.max(np.abs(rx))
    assert np.all(np.abs(gx - rx) <= 4 * U * np.abs(rx) + 1e-6 * scale), np.max(np.abs(gx - rx)) / scale
    assert np.all(np.abs(gp - rp) <= 1e-5 * np.abs(rp) + 1e-7 * np.max(np.abs(rp))), (gp, rp)
    J = (N + period - 1) // period
    assert np.all(ge[:, J:] == 0.0)
    es = np.max(np.abs(re[:, :J]))
    assert np.all(np.abs(ge[:, :J] - re[:, :J]) <= 1e-5 * np.abs(re[:, :J]) + 1e-7 * es)


def test_backward_ragged_short_segment_tails(V):
    """Ragged voices whose last lane segment (50 samples at period 100) holds
    1, 2 or 3 samples, or a few whole segments: the adjoint's peeled first
    and last samples of a segment, against the oracle voice by voice."""
    lens = [1, 2, 3, 51, 52, 53, 101, 150, 3201, 3202, 6403]
    B, N = len(lens), max(lens)
    x, env, params = _inputs(B, N, 17)
    w = np.random.default_rng(18).standard_normal((B, N)).astype(np.float32)
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    xp = torch.from_numpy(np.concatenate([x[b, :l] for b, l in enumerate(lens)])).cuda()
    wp = torch.from_numpy(np.concatenate([w[b, :l] for b, l in enumerate(lens)])).cuda()
    E, P = torch.from_numpy(env).cuda(), torch.from_numpy(params).cuda()
    O = torch.from_numpy(offs).cuda()
    _, st = V.lowpass(xp, E, P, 100, SR, offsets=O, max_samples=N, keep_states=True)
    gx, gp, ge = V.lowpass_backward(xp, wp, E, P, st, 100, SR, offsets=O, max_samples=N)
    gx, gp, ge = gx.cpu().numpy(), gp.cpu().numpy(), ge.cpu().numpy()
    for b, l in enumerate(lens):
        rx, rp, re = _oracle_grads(x[b:b + 1, :l], env[b:b + 1], params[b:b + 1], w[b:b + 1, :l])
        got = gx[offs[b]:offs[b + 1]]
        scale = np.max(np.abs(rx))
        assert np.all(np.abs(got - rx[0]) <= 4 * U * np.abs(rx[0]) + 1e-6 * scale), (b, l)
        assert np.all(np.abs(gp[b] - rp[0]) <= 1e-5 * np.abs(rp[0]) + 1e-7 * np.max(np.abs(rp))), (b, l)
        J = (l + 99) // 100
        es = np.max(np.abs(re[0, :J]))
        assert np.all(np.abs(ge[b, :J] - re[0, :J]) <= 1e-5 * np.abs(re[0, :J]) + 1e-7 * es), (b, l)


def test_adjoint_identity_at_full_size(V):
    """<dL/dx, dx> = <g, H dx> for the linear map H = lowpass(., env, params)
    on the ragged 16384-voice batch (1, 2, 4 s)."""
    B = 16384
    lens = np.array([44100, 88200, 176400])[np.arange(B) % 3]
    offs = torch.from_numpy(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)).cuda()
    total = int(lens.sum())
    gen = torch.Generator(device="cuda").manual_seed(0)
    dx = torch.randn(total, device="cuda", generator=gen)
    g = torch.randn(total, device="cuda", generator=gen)
    J = 1764
    env = torch.rand(B, J, device="cuda", generator=gen)
    params = torch.stack([torch.rand(B, device="cuda", generator=gen) * 70 + 30,
                          torch.rand(B, device="cuda", generator=gen) * 72 - 24,
                          torch.rand(B, device="cuda", generator=gen) * 14.5 + 0.5], 1).contiguous()
    hx, st = V.lowpass(dx, env, params, 100, SR, offsets=offs, max_samples=176400, keep_states=True)
    gx, gp, ge = V.lowpass_backward(dx, g, env, params, st, 100, SR, offsets=offs, max_samples=176400)
    lhs = float(torch.dot(gx.double(), dx.double()))
    rhs = float(torch.dot(g.double(), hx.double()))
    assert abs(lhs - rhs) <= 1e-5 * (float(gx.double().abs().dot(dx.double().abs())) + 1.0)
    assert torch.isfinite(gp).all() and torch.isfinite(ge).all()
    # the launch order (longest voices first, as timed) changes no result
    order = torch.from_numpy(np.argsort(-lens, kind="stable").astype(np.int32)).cuda()
    hx2, st2 = V.lowpass(dx, env, params, 100, SR, offsets=offs, max_samples=176400,
                         keep_states=True, order=order)
    gx2, gp2, ge2 = V.lowpass_backward(dx, g, env, params, st2, 100, SR, offsets=offs,
                                       max_samples=176400, order=order)
    assert torch.equal(hx2, hx)           # (rows of st past a voice's chunks are unwritten)
    assert torch.equal(gx2, gx) and torch.equal(gp2, gp) and torch.equal(ge2, ge)
    # sampled voices of each length against the oracle (forward)
    for b in (0, 1, 2):
        s, e = int(offs[b]), int(offs[b + 1])
        ref = _ref(dx[s:e].cpu().numpy()[None], env[b:b + 1].cpu().numpy(),
                   params[b:b + 1].cpu().numpy())[0]
        _check_y(hx[s:e].cpu().numpy(), ref)


def test_autograd_function_and_errors(V):
    x, env, params = _inputs(2, 1000, 3)
    X = torch.from_numpy(x).cuda().requires_grad_()
    E = torch.from_numpy(env).cuda().requires_grad_()
    P = torch.from_numpy(params).cuda().requires_grad_()
    w = torch.randn(2, 1000, device="cuda")
    (V.LowPass.apply(X, E, P) * w).sum().backward()
    rx, rp, re = _oracle_grads(x, env, params, w.cpu().numpy())
    assert np.allclose(X.grad.cpu().numpy(), rx, rtol=1e-5, atol=1e-6 * np.max(np.abs(rx)))
    assert np.allclose(P.grad.cpu().numpy(), rp, rtol=1e-5, atol=1e-7 * np.max(np.abs(rp)))
    L = V.lib()
    y = torch.empty_like(X)
    s = torch.cuda.current_stream().cuda_stream
    args = lambda period, env_ld: (X.data_ptr(), None, 2, 1000, 1000, E.data_ptr(), env_ld,
                                   P.data_ptr(), period, SR, y.data_ptr(), None, 0, None, s)
    assert L.synth_vcf_lowpass(*args(3, E.shape[1])) == -4          # period 3: unsupported
    assert L.synth_vcf_lowpass(*args(100, 9)) == -1                 # env rows too short
    assert L.synth_vcf_lowpass(*args(100, E.shape[1])) == 0
    assert L.synth_vcf_lowpass_backward(X.data_ptr(), y.data_ptr(), None, 2, 1000, 1000,
                                        E.data_ptr(), E.shape[1], P.data_ptr(), 100, SR, None, 0,
                                        y.data_ptr(), P.data_ptr(), None, None, s) == -1   # no states
