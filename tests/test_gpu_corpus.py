"""The corpus generator (synth_generate through paper_2104_12922_amd.corpus):
voices addressed by global index g, against the oracle (parameters bit-exact,
audio within 1e-4, the test-split flag), across a test-block boundary and at
large indices; shards and arbitrary index lists give bitwise the voices of a
single contiguous batch."""
import numpy as np
import pytest
import torch

import workloads as W
from oracle import philox, voice

pytestmark = pytest.mark.gpu
TOL = 1e-4


@pytest.fixture(scope="module")
def corpus():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    from paper_2104_12922_amd import corpus
    return corpus


def oracle(seed, ids, n):
    ids = np.asarray(ids, dtype=np.uint64)
    u = philox.sample_params(seed, ids)
    y = voice.render_uniform(torch.tensor(u), ids, n, W.default_nebula().table(), noise_seed=seed)
    return u, y.numpy(), np.array([voice.is_test(int(g)) for g in ids])


@pytest.mark.parametrize("seed,first_g,count,n", [(0, 9213, 6, 176400), (7, 2**40 + 5118, 5, 44100)])
def test_batch_matches_oracle_across_a_test_block_boundary(corpus, seed, first_g, count, n):
    gen = corpus.Synth1B1(W.default_nebula().table(), seed=seed, n_samples=n)
    audio, params, is_test = gen.batch(first_g, count)
    torch.cuda.synchronize()
    u, y, t = oracle(seed, np.arange(count, dtype=np.uint64) + np.uint64(first_g), n)
    assert np.array_equal(params.cpu().numpy().astype(np.float64), u)
    assert np.array_equal(is_test.cpu().numpy(), t) and t.any() and (~t).any()
    assert np.abs(audio.cpu().numpy().astype(np.float64) - y).max() <= TOL


def test_shards_and_index_lists_are_bitwise_the_contiguous_batch(corpus):
    tab = W.default_nebula().table()
    first, count, n = 9000, 700, 22050
    whole = corpus.Synth1B1(tab, seed=3, n_samples=n, batch_size=count).batch(first, count)
    rows = {}
    for r in range(3):
        gen = corpus.Synth1B1(tab, seed=3, n_samples=n, batch_size=64, rank=r, world=3)
        for g0, a, p, t in gen.stream(first, count):
            for i in range(a.shape[0]):
                assert g0 + i not in rows
                rows[g0 + i] = (a[i], p[i], t[i])
    assert sorted(rows) == list(range(first, first + count))
    for g, (a, p, t) in rows.items():
        i = g - first
        assert torch.equal(a, whole[0][i]) and torch.equal(p, whole[1][i]) and bool(t == whole[2][i])
    gen = corpus.Synth1B1(tab, seed=3, n_samples=n)
    pick = torch.tensor([9699, 9001, 9216, 9215, 9500], dtype=torch.int64, device="cuda")
    a, p, t = gen.voices(pick)
    for k, g in enumerate(pick.tolist()):
        assert torch.equal(a[k], whole[0][g - first]) and torch.equal(p[k], whole[1][g - first])
    test_rows = [(g0, a, p, t) for g0, a, p, t in gen.stream(first, count, split="test")]
    assert test_rows and all(bool(t.all()) for _, _, _, t in test_rows)
    assert sum(int(t.numel()) for _, _, _, t in test_rows) == int(whole[2].sum())
