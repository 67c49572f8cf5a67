"""The allocation-free render entry point (synth_render_noalloc), called
through the C ABI, against synth_render_ws (the same plan with a caller
workspace): bit-identical audio on two calls in a row, the second with a
smaller batch and length, and SYNTH_ENOMEM beyond the static array's size."""
import ctypes

import numpy as np
import pytest
import torch

import workloads as W

pytestmark = pytest.mark.gpu
ENOMEM = -2


@pytest.fixture(scope="module")
def S():
    if not torch.cuda.is_available():
        pytest.skip("needs a GPU")
    import paper_2104_12922_amd as S
    return S


def noalloc(S, u, table, n, seed, first_g=0):
    from paper_2104_12922_amd import _native
    L = _native.lib()
    cfg, keep = _native.make_config(table, noise_seed=seed)
    out = torch.full((u.shape[0], n), float("nan"), device="cuda")
    st = L.synth_render_noalloc(ctypes.byref(cfg), u.data_ptr(), None, first_g, u.shape[0], None, n,
                                out.data_ptr(), torch.cuda.current_stream().cuda_stream)
    _native.check("synth_render_noalloc", st)
    return out


def test_noalloc_render_matches_workspace_render_twice(S):
    from paper_2104_12922_amd import _native
    tab = W.default_nebula().table()
    L = _native.lib()
    for B, n, seed, first_g in ((128, 176400, 0, 0), (37, 66150, 5, 1000)):
        cfg, keep = _native.make_config(tab, noise_seed=seed)
        assert L.synth_render_workspace(ctypes.byref(cfg), B, n) > 0     # a split plan with carries
        u = S.synth_sample_params(seed, first_g, B)
        got = noalloc(S, u, tab, n, seed, first_g)
        ref = S.synth_render(u, tab, n_samples=n, noise_seed=seed, first_g=first_g)   # synth_render_ws
        torch.cuda.synchronize()
        assert torch.equal(got, ref), (B, n)


def test_noalloc_rejects_batches_beyond_the_scratch_size(S):
    from paper_2104_12922_amd import _native
    tab = W.default_nebula().table()
    L = _native.lib()
    cfg, keep = _native.make_config(tab)
    B, n = 1000, 44100 * 600                           # 1000 x 10 min: 136 MB of carries
    assert L.synth_render_workspace(ctypes.byref(cfg), B, n) > (16 << 20)
    u = torch.zeros(1, 78, device="cuda")
    out = torch.zeros(1, device="cuda")
    st = L.synth_render_noalloc(ctypes.byref(cfg), u.data_ptr(), None, 0, B, None, n, out.data_ptr(),
                                torch.cuda.current_stream().cuda_stream)
    assert st == ENOMEM
