"""Four-operator FM voice on the GPU against the float64 oracle
(oracle/fm.py), through the C ABI.

Bound: the kernel's float32 sine (hardware, revolutions, absolute error
within EPS of the float64 sine of the reduced phase) and float32 modulation
sums make each operator's output err by EPS plus 2 pi |M| times its
modulators' errors, so with A_3 = 1, A_i = 1 + 2 pi sum_{j > i} |M_ij| L_j A_j
(L_j: operator j's level) a sample errs by at most EPS sum_i w_i L_i A_i /
max(1, sum w)."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import fm as OFM
from oracle import philox
from oracle.voice import map_params

pytestmark = pytest.mark.gpu

EPS = 4e-6
PAIRS = OFM.PAIRS


@pytest.fixture(scope="module")
def F():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2104_12922_amd import fm
    return fm


def _bound(u, table):
    v = map_params(torch.tensor(u, dtype=torch.float64), table).numpy()
    B = v.shape[0]
    A = np.ones((B, 4))
    L = np.stack([v[:, b + 2] for b in OFM.OP_BASE], 1)
    M = np.zeros((B, 4, 4))
    for k, (i, j) in enumerate(PAIRS):
        M[:, i, j] = np.abs(v[:, OFM.MOD_BASE + k])
    for i in (2, 1, 0):
        A[:, i] = 1 + 2 * np.pi * sum(M[:, i, j] * L[:, j] * A[:, j] for j in range(i + 1, 4))
    w = v[:, OFM.MIX_BASE:OFM.MIX_BASE + 4]
    return EPS * (w * L * A).sum(1) / np.maximum(1.0, w.sum(1))


def test_draw_matches_oracle(F):
    ids = torch.tensor([0, 1, 77, 2 ** 40 + 9], dtype=torch.int64, device="cuda")
    got = F.fm_sample_params(5, voice_ids=ids).cpu().numpy().astype(np.float64)
    ref = OFM.sample_params(5, ids.cpu().numpy().astype(np.uint64))
    assert np.array_equal(got, ref)
    got2 = F.fm_sample_params(5, first_g=10, batch=3).cpu().numpy().astype(np.float64)
    assert np.array_equal(got2, OFM.sample_params(5, np.arange(10, 13, dtype=np.uint64)))


@pytest.mark.parametrize("B,N", [(6, 13000), (3, 6401), (4, 7), (2, 44100)])
def test_render_matches_oracle(F, B, N):
    tab = W.fm_default_nebula().table()
    u = F.fm_sample_params(11 + N, batch=B)
    y = F.fm_render(u, tab, n_samples=N).cpu().numpy()
    ref = OFM.render_uniform(torch.tensor(u.cpu().numpy().astype(np.float64)), N, tab).numpy()
    bnd = _bound(u.cpu().numpy().astype(np.float64), tab)
    err = np.abs(y - ref).max(1)
    assert np.all(err <= bnd), (err, bnd)


def test_ragged_and_silent_tail(F):
    tab = W.fm_default_nebula(duration_min=0.1).table()
    tab[1, 1] = 0.5                                   # short notes: long silent tails
    for b in OFM.OP_BASE:
        tab[b + 6, 1] = 0.2                           # releases up to 0.2 s
    lens = [0, 1, 5, 99, 100, 101, 6400, 6401, 44100, 88203]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    u = F.fm_sample_params(3, batch=len(lens))
    y = F.fm_render(u, tab, offsets=torch.from_numpy(offs).cuda()).cpu().numpy()
    uu = u.cpu().numpy().astype(np.float64)
    ref = OFM.render(torch.tensor(uu), lens, tab).numpy()
    bnd = _bound(uu, tab)
    for b, l in enumerate(lens):
        s, e = offs[b], offs[b + 1]
        assert np.all(np.abs(y[s:e] - ref[s:e]) <= bnd[b])
    # the 2 s voice ends in exact silence (note <= 0.5 s, release <= 0.2 s)
    assert np.all(y[offs[-2] + 44100:offs[-1]] == 0.0)


def test_full_size_sampled(F):
    """The ragged 16384-voice workload shape (1, 2, 4 s): sampled voices
    against the oracle, and the whole batch finite and bounded."""
    B = 16384
    lens = np.array([44100, 88200, 176400])[np.arange(B) % 3]
    offs = torch.from_numpy(np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)).cuda()
    tab = W.fm_default_nebula(duration_min=0.1).table()
    u = F.fm_sample_params(0, batch=B)
    y = F.fm_render(u, tab, offsets=offs)
    assert torch.isfinite(y).all() and float(y.abs().max()) <= 1.0 + 1e-6
    # the launch order (longest voices first, as timed) changes no sample
    order = torch.from_numpy(np.argsort(-lens, kind="stable").astype(np.int32)).cuda()
    assert torch.equal(F.fm_render(u, tab, offsets=offs, order=order), y)
    uu = u.cpu().numpy().astype(np.float64)
    for b in (0, 1, 2, 12345):
        s, e = int(offs[b]), int(offs[b + 1])
        ref = OFM.render_uniform(torch.tensor(uu[b:b + 1]), e - s, tab).numpy()[0]
        assert np.max(np.abs(y[s:e].cpu().numpy() - ref)) <= _bound(uu[b:b + 1], tab)[0]


def test_errors(F):
    tab = W.fm_default_nebula().table()
    u = F.fm_sample_params(0, batch=2)
    bad = tab.copy()
    bad[5, 2] = 0.0                                    # curve 0
    with pytest.raises(Exception):
        F.fm_render(u, bad, n_samples=100)
    bad = tab.copy()
    bad[2 + 7, 0] = 0.0                                # envelope exponent minimum 0
    with pytest.raises(Exception):
        F.fm_render(u, bad, n_samples=100)
    with pytest.raises(Exception):
        F.fm_render(u, tab, n_samples=100, sample_rate=44100.0, control_rate=440.0)
    with pytest.raises(Exception):                     # period 98: not a multiple of 4
        F.fm_render(u, tab, n_samples=100, sample_rate=44100.0, control_rate=450.0)
    # other periods that are multiples of 4 (here 64 and 1024) render
    for sr, rc in ((44800.0, 700.0), (65536.0, 64.0)):
        y = F.fm_render(u, tab, n_samples=3000, sample_rate=sr, control_rate=rc).cpu().numpy()
        uu = u.cpu().numpy().astype(np.float64)
        ref = OFM.render_uniform(torch.tensor(uu), 3000, tab, sr=sr, rc=rc).numpy()
        assert np.all(np.abs(y - ref).max(1) <= _bound(uu, tab)), (sr, rc)
