"""Pairwise L1 sums and the MMD of sets of sounds (Section 5, equation "mmd")
on the GPU against the float64 oracle (oracle/mmd.py), through the C ABI.

Bound: each pair's distance is accumulated in float32 over runs of at most
256 dimensions (one rounding per difference and per addition), then in
float64, so |S_gpu - S| <= 257 u S + (float64 terms) with u = 2^-24, and the
MMD, a combination of three such sums, is off by at most 257 u (2 S_xy / nm +
S_xx / n^2 + S_yy / m^2).  Small-integer data make every float32 operation
exact, so there the results must be bit-identical to the oracle's."""

import numpy as np
import pytest
import torch

from oracle import mmd as OM

pytestmark = pytest.mark.gpu

U32 = 2.0 ** -24
RUN_BOUND = 257 * U32 + 1e-13


@pytest.fixture(scope="module")
def nb():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2104_12922_amd import nebula
    return nebula


def _gen(seed, n, dim, shift=0.0, scale=1.0):
    g = torch.Generator().manual_seed(seed)
    return (torch.randn(n, dim, generator=g) * scale + shift).float()


def _oracle(X, Y):
    Xd, Yd = X.double().numpy(), Y.double().numpy()
    sxy, sxx, syy = OM.l1_distance_sum(Xd, Yd), OM.l1_distance_sum(Xd, Xd), OM.l1_distance_sum(Yd, Yd)
    return OM.mmd(Xd, Yd), sxy, sxx, syy


def _check(got, X, Y):
    n, m = X.shape[0], Y.shape[0]
    mmd, sxy, sxx, syy = _oracle(X, Y)
    g = got.cpu().numpy()
    for a, b in ((g[1], sxy), (g[2], sxx), (g[3], syy)):
        assert abs(a - b) <= RUN_BOUND * b, (a, b)
    scale = 2 * sxy / (n * m) + sxx / (n * n) + syy / (m * m)
    assert abs(g[0] - mmd) <= RUN_BOUND * scale + 1e-15, (g[0], mmd, scale)
    return mmd


@pytest.mark.parametrize("n,m,dim", [(1, 1, 1), (1, 5, 3), (3, 5, 7), (64, 64, 32), (65, 63, 257),
                                     (100, 37, 1000), (130, 70, 8197), (7, 300, 513)])
def test_mmd_matches_oracle(nb, n, m, dim):
    X = _gen(n * 1000 + dim, n, dim)
    Y = _gen(m * 1000 + dim + 1, m, dim, shift=0.2, scale=1.3)
    got = nb.mmd_l1(X.cuda(), Y.cuda())
    mmd = _check(got, X, Y)
    if n > 1 or m > 1:
        assert mmd > 0.0 and float(got[0]) > 0.0


def test_small_integers_are_bit_exact(nb):
    g = torch.Generator().manual_seed(5)
    X = torch.randint(-8, 9, (70, 600), generator=g).float()
    Y = torch.randint(-6, 11, (130, 600), generator=g).float()
    got = nb.mmd_l1(X.cuda(), Y.cuda()).cpu().numpy()
    mmd, sxy, sxx, syy = _oracle(X, Y)
    assert got[1] == sxy and got[2] == sxx and got[3] == syy
    assert got[0] == mmd


def test_identity_symmetry_determinism(nb):
    X = _gen(1, 90, 700).cuda()
    Y = _gen(2, 50, 700, shift=0.5).cuda()
    assert float(nb.mmd_l1(X, X)[0]) == 0.0                 # exactly: S(X, X) as S(X, Y = X)
    a = nb.mmd_l1(X, Y).cpu().numpy()
    b = nb.mmd_l1(X, Y).cpu().numpy()
    assert np.array_equal(a, b)                             # fixed summation order
    c = nb.mmd_l1(Y, X).cpu().numpy()
    assert abs(c[1] - a[1]) <= 2 * RUN_BOUND * a[1]
    assert c[2] == a[3] and c[3] == a[2]
    assert abs(c[0] - a[0]) <= 2 * RUN_BOUND * (2 * a[1] / (90 * 50) + a[2] / 8100 + a[3] / 2500)


def test_strided_and_empty_inputs(nb):
    dim = 333
    wide = _gen(3, 80, dim + 13).cuda()
    A = wide[:, 5:5 + dim]                                  # row stride dim + 13, unaligned rows
    B = _gen(4, 41, dim).cuda()
    s1 = float(nb.l1_pair_sum(A, B))
    s2 = float(nb.l1_pair_sum(A.contiguous(), B))
    assert s1 == s2                                         # same arithmetic, other load path
    assert abs(s1 - OM.l1_distance_sum(A.cpu().double().numpy(), B.cpu().double().numpy())) <= RUN_BOUND * s1
    assert float(nb.l1_pair_sum(A[:0], B)) == 0.0
    assert float(nb.l1_pair_sum(A, B[:0])) == 0.0
    assert float(nb.l1_pair_sum(A[:, :0], B[:, :0])) == 0.0
    with pytest.raises(ValueError):
        nb.mmd_l1(A[:0].contiguous(), B)


def test_c_abi_errors(nb):
    L = nb.lib()
    X = torch.zeros(10, 8, device="cuda")
    out = torch.zeros(4, dtype=torch.float64, device="cuda")
    need = L.synth_mmd_l1_workspace(10, 10, 8)
    assert need > 0
    ws = torch.empty(need, dtype=torch.uint8, device="cuda")
    s = torch.cuda.current_stream().cuda_stream
    SYNTH_EINVAL, SYNTH_ENOMEM = -1, -2
    assert L.synth_mmd_l1(X.data_ptr(), 10, X.data_ptr(), 10, 8, ws.data_ptr(), need - 8,
                          out.data_ptr(), s) == SYNTH_ENOMEM
    assert L.synth_mmd_l1(X.data_ptr(), 0, X.data_ptr(), 10, 8, ws.data_ptr(), need,
                          out.data_ptr(), s) == SYNTH_EINVAL
    assert L.synth_mmd_l1(X.data_ptr(), 10, X.data_ptr(), 10, 8, ws.data_ptr() + 4, need,
                          out.data_ptr(), s) == SYNTH_EINVAL
    assert L.synth_l1_pair_sum(X.data_ptr(), 7, 10, X.data_ptr(), 8, 10, 8, ws.data_ptr(), need,
                               out.data_ptr(), s) == SYNTH_EINVAL           # lda < dim
    assert L.synth_l1_pair_sum_workspace(1 << 18, 4, 8) == 0                # beyond 2^17 sounds
    assert L.synth_mmd_l1(X.data_ptr(), 10, X.data_ptr(), 10, 8, ws.data_ptr(), need,
                          out.data_ptr(), s) == 0
    torch.cuda.synchronize()
    assert float(out[0]) == 0.0


def test_paper_trial_size_sampled(nb):
    """n = m = 1000 sounds of 8192 features (the paper's MMD trials): row
    blocks against the oracle, and additivity over row blocks at full size."""
    n, dim = 1000, 8192
    X = _gen(11, n, dim).cuda()
    Y = _gen(12, n, dim, shift=0.05).cuda()
    full = nb.mmd_l1(X, Y).cpu().numpy()
    parts = sum(float(nb.l1_pair_sum(X[i:i + 250], Y)) for i in range(0, n, 250))
    assert abs(parts - full[1]) <= 2 * RUN_BOUND * full[1]
    for (i0, i1, j0, j1) in ((0, 24, 0, 16), (487, 530, 970, 1000), (999, 1000, 0, 1000)):
        a, b = X[i0:i1], Y[j0:j1]
        got = float(nb.l1_pair_sum(a, b))
        ref = OM.l1_distance_sum(a.cpu().double().numpy(), b.cpu().double().numpy())
        assert abs(got - ref) <= RUN_BOUND * ref
    assert full[0] > 0.0


def test_logmel_sets_of_renders(nb):
    """Embeddings of real renders: log-mel features of 1 s voices drawn from
    the default nebula and from a curved one."""
    import workloads as W
    from paper_2104_12922_amd.nebula import SoundSets
    sets = SoundSets(n_sounds=48, n_samples=44100, seed=30)
    Xa = sets.embed(W.default_nebula().table(), 0).clone()
    Xb = sets.embed(W.curved_test_nebula().table(), 1).clone()
    Xc = sets.embed(W.default_nebula().table(), 2).clone()
    far = _check(nb.mmd_l1(Xa, Xb), Xa.cpu(), Xb.cpu())
    near = _check(nb.mmd_l1(Xa, Xc), Xa.cpu(), Xc.cpu())
    assert 0.0 < near < far          # two draws of one nebula are closer than two nebulas
