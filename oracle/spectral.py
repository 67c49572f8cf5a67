"""Spectral features and losses on rendered audio (float64, torch CPU).

TEST INFRASTRUCTURE ONLY (see ``oracle/__init__``).

The paper scores sounds with a multi-scale spectrogram distance, linear plus
log magnitudes over several FFT sizes, and prefers L1 distances (Section 4.3,
Table "distance-eval").  The loss used here for gradient-based sound matching
is its log-magnitude L1 form at three resolutions; the learned proposal reads
log-mel features.  Where the paper leaves details open, the readings taken
here are: no centring or padding, a periodic Hann window, the HTK mel scale.

  frames(x, n, hop)   F = floor((N - n) / hop) + 1 frames, frame t starts at t*hop
  stft(x, n, hop)     X[t, k] = sum_m w(m) x(t*hop + m) exp(-2 pi i k m / n),
                      k = 0..n/2, w(m) = (1 - cos(2 pi m / n)) / 2
  mrstft_loss(x, T)   sum over n in (512, 1024, 2048), hop n/4, of the mean over
                      (voice, frame, bin) of |log(|X| + 1e-5) - log(|T| + 1e-5)|;
                      a resolution without a complete frame contributes 0
  logmel(x)           log(M |X|^2 + 1e-6), 64 frames of n = 2048 at hop 2756,
                      128 HTK triangles from 0 to sr/2, no area normalisation
"""
from __future__ import annotations

import math

import numpy as np
import torch

F64 = torch.float64
MR_SIZES = (512, 1024, 2048)
MAG_EPS = 1e-5
MEL_EPS = 1e-6
MEL_BINS = 128
MEL_FRAMES = 64
MEL_NFFT = 2048
MEL_HOP = 2756


def hann(n: int) -> torch.Tensor:
    """Periodic Hann window of length n."""
    m = torch.arange(n, dtype=F64)
    return 0.5 - 0.5 * torch.cos(2.0 * math.pi * m / n)


def num_frames(N: int, n: int, hop: int) -> int:
    return 0 if N < n else (N - n) // hop + 1


def frames(x: torch.Tensor, n: int, hop: int, count: int | None = None) -> torch.Tensor:
    """[..., N] -> [..., F, n] frames starting at t * hop (no padding)."""
    F = num_frames(x.shape[-1], n, hop) if count is None else count
    idx = torch.arange(F)[:, None] * hop + torch.arange(n)[None, :]
    return x[..., idx]


def stft(x: torch.Tensor, n: int, hop: int, count: int | None = None) -> torch.Tensor:
    """One-sided STFT [..., F, n/2 + 1] (complex128) via the FFT as a library step."""
    return torch.fft.rfft(frames(x, n, hop, count) * hann(n), dim=-1)


def dft_bruteforce(frame: np.ndarray) -> np.ndarray:
    """Direct O(n^2) DFT of one windowed frame, bins 0..n/2 (pins ``stft``)."""
    n = len(frame)
    k = np.arange(n // 2 + 1)[:, None]
    m = np.arange(n)[None, :]
    return (frame[None, :] * np.exp(-2j * np.pi * k * m / n)).sum(-1)


def mrstft_loss(x: torch.Tensor, target: torch.Tensor, sizes=MR_SIZES) -> torch.Tensor:
    """Multi-resolution log-magnitude STFT L1 between [B, N] batches (scalar).
    A resolution with no complete frame (N < n) contributes 0."""
    total = torch.zeros((), dtype=F64)
    for n in sizes:
        if num_frames(x.shape[-1], n, n // 4) == 0:
            continue
        X = stft(x, n, n // 4).abs()
        T = stft(target, n, n // 4).abs()
        total = total + (torch.log(X + MAG_EPS) - torch.log(T + MAG_EPS)).abs().mean()
    return total


def mrstft_loss_per_voice(x: torch.Tensor, target: torch.Tensor, sizes=MR_SIZES) -> torch.Tensor:
    """Same loss, one value per voice [B] (mean over frames and bins of each voice)."""
    total = torch.zeros(x.shape[0], dtype=F64)
    for n in sizes:
        if num_frames(x.shape[-1], n, n // 4) == 0:
            continue
        X = stft(x, n, n // 4).abs()
        T = stft(target, n, n // 4).abs()
        total = total + (torch.log(X + MAG_EPS) - torch.log(T + MAG_EPS)).abs().mean(dim=(-2, -1))
    return total


def hz_to_mel(f):
    return 2595.0 * np.log10(1.0 + np.asarray(f, dtype=np.float64) / 700.0)


def mel_to_hz(m):
    return 700.0 * (10.0 ** (np.asarray(m, dtype=np.float64) / 2595.0) - 1.0)


def mel_filterbank(sr: float = 44100.0, n_fft: int = MEL_NFFT, n_mels: int = MEL_BINS) -> np.ndarray:
    """[n_mels, n_fft/2 + 1] HTK triangles: n_mels + 2 edges equally spaced on the
    mel scale from 0 Hz to sr/2; filter b rises from edge b to edge b+1 and falls
    to edge b+2, with peak value 1 (no area normalisation)."""
    edges = mel_to_hz(np.linspace(hz_to_mel(0.0), hz_to_mel(sr / 2.0), n_mels + 2))
    f = np.arange(n_fft // 2 + 1) * sr / n_fft
    M = np.zeros((n_mels, len(f)))
    for b in range(n_mels):
        lo, c, hi = edges[b], edges[b + 1], edges[b + 2]
        up = (f - lo) / (c - lo)
        down = (hi - f) / (hi - c)
        M[b] = np.maximum(0.0, np.minimum(up, down))
    return M


def logmel(x: torch.Tensor, sr: float = 44100.0) -> torch.Tensor:
    """[B, N] -> [B, 128, 64] log-mel features (mel bin major, frame minor)."""
    X = stft(x, MEL_NFFT, MEL_HOP, count=MEL_FRAMES)           # [B, 64, 1025]
    P = X.real ** 2 + X.imag ** 2
    M = torch.from_numpy(mel_filterbank(sr))                    # [128, 1025]
    mel = torch.einsum("bk,ntk->nbt", M, P)                     # [B, 128, 64]
    return torch.log(mel + MEL_EPS)


def logmel_bf16(x: torch.Tensor, sr: float = 44100.0) -> torch.Tensor:
    """Log-mel with bfloat16 operands at fixed points: the frames (float32
    samples) rounded to bfloat16; the DFT basis with the periodic Hann window
    folded in, w(k) cos(2 pi f k / n) and -w(k) sin(2 pi f k / n), computed in
    float64, rounded to float32 and then to bfloat16; the power spectrum and the
    mel basis rounded to bfloat16; products accumulated in float64 here.
    Windowing the basis instead of the frame is the same linear map, so this
    differs from ``logmel`` only by the roundings.  Returns [B, 128, 64]."""
    n = MEL_NFFT
    k = torch.arange(n, dtype=F64)
    w = 0.5 - 0.5 * torch.cos(2.0 * math.pi * k / n)                  # float64 window
    fr = frames(x.float(), n, MEL_HOP, count=MEL_FRAMES)
    fr = fr.to(torch.bfloat16).to(F64)
    f = torch.arange(n // 2 + 1, dtype=torch.int64)[:, None]
    ph = (f * torch.arange(n)[None, :]) % n                           # exact angle reduction
    ang = 2.0 * math.pi * ph.to(F64) / n
    cosb = (w * torch.cos(ang)).float().to(torch.bfloat16).to(F64)
    sinb = (-w * torch.sin(ang)).float().to(torch.bfloat16).to(F64)
    re = fr @ cosb.T
    im = fr @ sinb.T
    P = (re * re + im * im).float().to(torch.bfloat16).to(F64)        # [B, 64, 1025]
    M = torch.from_numpy(mel_filterbank(sr)).float().to(torch.bfloat16).to(F64)
    mel = torch.einsum("bk,ntk->nbt", M, P)
    return torch.log(mel + MEL_EPS)


def logmel_p16(x: torch.Tensor, sr: float = 44100.0) -> torch.Tensor:
    """Log-mel with the power spectrum and the mel basis rounded to bfloat16:
    the windowed frames are formed in float32 (window and samples float32),
    transformed exactly (float64 FFT), |X|^2 rounded through float32 to
    bfloat16, projected with the bfloat16 mel basis in float64, log(+1e-6).
    Returns [B, 128, 64]."""
    n = MEL_NFFT
    k = torch.arange(n, dtype=torch.float32)
    w = 0.5 - 0.5 * torch.cos(2.0 * math.pi * k / n)                  # float32 window
    fr = (frames(x.float(), n, MEL_HOP, count=MEL_FRAMES) * w).to(F64)
    X = torch.fft.rfft(fr, dim=-1)                                    # [B, 64, 1025]
    P = (X.real ** 2 + X.imag ** 2).float().to(torch.bfloat16).to(F64)
    M = torch.from_numpy(mel_filterbank(sr)).float().to(torch.bfloat16).to(F64)
    mel = torch.einsum("bk,ntk->nbt", M, P)
    return torch.log(mel + MEL_EPS)
