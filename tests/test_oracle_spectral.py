"""Pins of the spectral oracle: brute-force DFT, Parseval, pure-tone peaks,
closed-form loss values, mel filterbank invariants."""
import math

import numpy as np
import pytest
import torch

from oracle import spectral as sp

F64 = torch.float64


def test_frame_counts_match_the_configured_resolutions():
    assert [sp.num_frames(176400, n, n // 4) for n in (512, 1024, 2048)] == [1375, 686, 341]
    assert sp.num_frames(176400, 2048, 2756) == 64
    assert sp.num_frames(100, 512, 128) == 0


def test_stft_matches_bruteforce_dft():
    rng = np.random.default_rng(0)
    x = torch.tensor(rng.standard_normal((2, 3000)))
    X = sp.stft(x, 256, 64).numpy()
    w = sp.hann(256).numpy()
    for b in range(2):
        for t in (0, 5, X.shape[1] - 1):
            ref = sp.dft_bruteforce(x[b, t * 64:t * 64 + 256].numpy() * w)
            assert np.abs(X[b, t] - ref).max() < 1e-10


def test_hann_is_periodic_and_parseval_holds():
    w = sp.hann(8).numpy()
    assert np.allclose(w, [0, 0.1464466, 0.5, 0.8535534, 1, 0.8535534, 0.5, 0.1464466], atol=1e-7)
    rng = np.random.default_rng(1)
    fr = rng.standard_normal(512)
    X = np.fft.fft(fr * sp.hann(512).numpy())
    Xh = sp.stft(torch.tensor(fr)[None], 512, 512)[0, 0].numpy()
    assert np.allclose(Xh, X[:257], atol=1e-10)
    # Parseval on the full spectrum rebuilt from the one-sided one
    full = np.sum(np.abs(Xh) ** 2) * 2 - np.abs(Xh[0]) ** 2 - np.abs(Xh[-1]) ** 2
    assert math.isclose(full / 512, np.sum((fr * sp.hann(512).numpy()) ** 2), rel_tol=1e-12)


def test_pure_tone_peaks_at_its_bin():
    sr, n = 44100.0, 2048
    k0 = 93
    f = k0 * sr / n
    t = np.arange(20000) / sr
    x = torch.tensor(np.sin(2 * np.pi * f * t))[None]
    X = sp.stft(x, n, n // 4).abs()[0]
    assert (X.argmax(-1) == k0).all()
    # periodic Hann: a bin-centred tone spreads over k0 +- 1 only, with a 1 : 1/2 ratio
    assert np.allclose((X[:, k0 + 1] / X[:, k0]).numpy(), 0.5, atol=1e-9)
    assert float(X[:, k0 + 3].max()) < 1e-9 * float(X[:, k0].max())


def test_mrstft_loss_closed_forms():
    rng = np.random.default_rng(2)
    x = torch.tensor(rng.standard_normal((3, 8000)))
    assert float(sp.mrstft_loss(x, x)) == 0.0
    # scaling by c: every |X| scales by c, so each term is |log c| up to the 1e-5 offset
    c = 3.0
    L = float(sp.mrstft_loss(c * x, x))
    assert abs(L - 3 * math.log(c)) < 1e-4
    assert math.isclose(float(sp.mrstft_loss(x, c * x)), L, rel_tol=0, abs_tol=1e-4)
    per = sp.mrstft_loss_per_voice(c * x, x)
    assert torch.allclose(per.mean(), torch.tensor(L, dtype=F64), atol=1e-12)
    # silence vs silence: log(1e-5) on both sides
    z = torch.zeros(1, 4096, dtype=F64)
    assert float(sp.mrstft_loss(z, z)) == 0.0


def test_mel_filterbank_invariants():
    M = sp.mel_filterbank()
    assert M.shape == (128, 1025)
    assert M.min() >= 0 and M.max() <= 1 + 1e-12
    f = np.arange(1025) * 44100 / 2048
    edges = sp.mel_to_hz(np.linspace(0, sp.hz_to_mel(22050), 130))
    # overlapping HTK triangles sum to exactly 1 between the first and last centre
    inside = (f >= edges[1]) & (f <= edges[-2])
    assert np.allclose(M[:, inside].sum(0), 1.0, atol=1e-12)
    # the mel scale: 1000 Hz ~ 1000 mel
    assert abs(sp.hz_to_mel(1000.0) - 1000.0) < 0.1
    assert np.allclose(sp.mel_to_hz(sp.hz_to_mel([10.0, 440.0, 8000.0])), [10.0, 440.0, 8000.0])


def test_logmel_shape_and_tone_bin():
    sr = 44100.0
    t = np.arange(176400) / sr
    f0 = 1000.0
    x = torch.tensor(np.sin(2 * np.pi * f0 * t))[None]
    L = sp.logmel(x)
    assert L.shape == (1, 128, 64)
    edges = sp.mel_to_hz(np.linspace(0, sp.hz_to_mel(22050), 130))
    expect = int(np.argmin(np.abs(edges[1:-1] - f0)))
    assert abs(int(L[0, :, 10].argmax()) - expect) <= 1
    z = sp.logmel(torch.zeros(1, 176400, dtype=F64))
    assert torch.allclose(z, torch.full_like(z, math.log(1e-6)))
