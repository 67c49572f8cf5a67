"""Learned proposal (inverse synthesis, audio -> parameters): log-mel features
and an MLP 8192 -> 1024 -> 1024 -> 78 (GELU, sigmoid output), trained with Adam.

Argument marshalling only: the DFT and mel GEMMs, the MLP forward and
backward GEMMs with their fused epilogues, the loss gradient, the bias and
statistics reductions and Adam all run in libsynth.so's HIP kernels.  bf16
tensors are torch.bfloat16 (raw bfloat16 storage, as the C ABI expects).
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _native
from . import _dev_ptr, _stream

BF16 = torch.bfloat16
F32 = torch.float32
MEL_FEATURES = 128 * 64


def _sig(L):
    vp, i64, i32, f32, sz = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int, ctypes.c_float, ctypes.c_size_t
    L.synth_gemm_bf16.argtypes = [i32, i32, i64, i64, i64, vp, i64, vp, i64, vp, i64, i32, vp, i32,
                                  vp, vp, f32, f32, vp]
    L.synth_logmel_workspace.restype = sz
    L.synth_logmel_workspace.argtypes = [i64]
    L.synth_logmel_init.argtypes = [ctypes.c_double, vp, vp, vp]
    L.synth_logmel.argtypes = [vp, vp, i64, i64, vp, vp, sz, vp, vp]
    L.synth_logmel_mfma.argtypes = [vp, vp, i64, i64, vp, vp, vp, sz, vp, vp]
    L.synth_logmel_standardized.argtypes = [vp, vp, i64, i64, vp, vp, vp, vp, vp, vp]
    L.synth_colstats.argtypes = [vp, i32, i64, i64, i64, vp, vp, vp]
    L.synth_standardize.argtypes = [vp, vp, vp, i64, i64, vp, vp]
    L.synth_feature_stats.argtypes = [vp, i64, i64, f32, vp, vp, vp]
    L.synth_to_bf16.argtypes = [vp, vp, i64, vp]
    L.synth_mlp_workspace.restype = sz
    L.synth_mlp_workspace.argtypes = [i64, i64, i64, i64]
    L.synth_mlp_forward.argtypes = [i64, i64, i64, i64] + [vp] * 13 + [sz, vp]
    L.synth_mlp_backward.argtypes = [i64, i64, i64, i64] + [vp] * 20 + [sz, vp]
    L.synth_adam.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
    L.synth_logit_init.argtypes = [vp, vp, vp, i64, f32, vp]
    L.synth_logit_adam.argtypes = [i64, vp, vp, vp, vp, vp, f32, f32, f32, f32, i32, vp]
    L.synth_best_update.argtypes = [vp, i64, i64, i64, i64, i64, vp, i64, vp, vp, vp, vp]
    f64 = ctypes.c_double
    L.synth_diff_reduce.argtypes = [i32, i32, vp, vp, i64, i64, i64, i64, f64, i32, vp, vp]
    L.synth_sum_f64.argtypes = [vp, i64, f64, vp, vp]
    L.synth_scale_rows.argtypes = [vp, vp, i64, i64, vp, vp]
    for n in ("synth_diff_reduce", "synth_sum_f64", "synth_scale_rows"):
        getattr(L, n).restype = ctypes.c_int
    for n in ("synth_gemm_bf16", "synth_logmel_init", "synth_logmel", "synth_logmel_mfma",
              "synth_colstats",
              "synth_standardize", "synth_to_bf16", "synth_mlp_forward", "synth_mlp_backward",
              "synth_adam", "synth_feature_stats", "synth_logit_init", "synth_logit_adam", "synth_best_update"):
        getattr(L, n).restype = ctypes.c_int
    return L


_L = None


def lib():
    global _L
    if _L is None:
        _L = _sig(_native.lib())
    return _L


def _p(t, name, dtype, numel=None):
    return _dev_ptr(t, name, dtype, numel)


def diff_reduce(a, b=None, kind=0, axis=1, scale=1.0, out=None, accumulate=False):
    """Fixed-order float64 sums of |a - b| (kind 0) or (a - b)^2 (kind 1) over
    the columns of each row (axis 1, out [rows]) or the rows of each column
    (axis 0, out [cols]), times scale (synth_diff_reduce)."""
    rows, cols = a.shape
    n_out = rows if axis == 1 else cols
    if out is None:
        out = torch.zeros(n_out, dtype=torch.float64, device=a.device)
    _native.check("synth_diff_reduce", lib().synth_diff_reduce(
        int(kind), int(axis), _p(a, "a", F32), _p(b, "b", F32, a.numel()) if b is not None else None,
        rows, cols, a.stride(0), b.stride(0) if b is not None else cols, float(scale),
        int(bool(accumulate)), _p(out, "out", torch.float64, n_out), _stream(a.device)))
    return out


def sum_f64(x, scale=1.0, out=None):
    """scale * sum(x) of a float64 device vector, in a fixed order (0-d float64)."""
    if out is None:
        out = torch.empty((), dtype=torch.float64, device=x.device)
    _native.check("synth_sum_f64", lib().synth_sum_f64(
        _p(x, "x", torch.float64), x.numel(), float(scale), _p(out, "out", torch.float64, 1),
        _stream(x.device)))
    return out


def scale_rows(g, s, out=None):
    """out[r, c] = g[r, c] * float(s[r]) (synth_scale_rows)."""
    rows, cols = g.shape
    if out is None:
        out = torch.empty_like(g)
    _native.check("synth_scale_rows", lib().synth_scale_rows(
        _p(g, "g", F32, rows * cols), _p(s, "s", torch.float64, rows),
        rows, cols, _p(out, "out", F32, rows * cols), _stream(g.device)))
    return out


def gemm_bf16(A, B, M, N, K, a_layout=0, b_layout=0, lda=None, ldb=None, out=None, out_bf16=False,
              bias=None, epilogue=0, aux=None, pre=None, alpha=1.0, beta=0.0):
    """C = epi(alpha A B + bias) (+ beta C) on the bf16 MFMA GEMM (see synth.h)."""
    lda = lda or (K if a_layout == 0 else M)
    ldb = ldb or (K if b_layout == 0 else N)
    if out is None:
        out = torch.empty(M, N, dtype=BF16 if out_bf16 else F32, device=A.device)
    ldc = out.shape[-1]
    _native.check("synth_gemm_bf16", lib().synth_gemm_bf16(
        a_layout, b_layout, M, N, K, _p(A, "A", BF16), lda, _p(B, "B", BF16), ldb,
        _p(out, "C", BF16 if out_bf16 else F32), ldc, int(out_bf16),
        _p(bias, "bias", F32) if bias is not None else None, epilogue,
        _p(aux, "aux", F32) if aux is not None else None,
        _p(pre, "pre", F32) if pre is not None else None, float(alpha), float(beta),
        _stream(A.device)))
    return out


class LogMel:
    """Log-mel features [B, 128 * 64] (mel-bin major) of renders.

    method "fft" (default): float32 FFT power spectrum; "mfma": the power
    spectrum as a bf16 DFT GEMM on the matrix cores."""

    def __init__(self, sample_rate: float = 44100.0, device="cuda", method: str = "fft"):
        if method not in ("fft", "mfma"):
            raise ValueError("method must be 'fft' or 'mfma'")
        self.device = torch.device(device)
        self.method = method
        self.dft = (torch.empty(2048, 2048, dtype=BF16, device=self.device)
                    if method == "mfma" else None)
        self.mel = torch.empty(128, 1032, dtype=BF16, device=self.device)
        _native.check("synth_logmel_init", lib().synth_logmel_init(
            float(sample_rate), self.dft.data_ptr() if self.dft is not None else None,
            self.mel.data_ptr(), _stream(self.device)))
        self._ws = None

    def standardized(self, audio: torch.Tensor, offsets: torch.Tensor, mean: torch.Tensor,
                     inv_std: torch.Tensor, out: torch.Tensor, rows: torch.Tensor | None = None):
        """bf16 standardised features of the ragged voices in one kernel
        (FFT method): voice b's row goes to out[rows[b]] (out[b] without
        rows); bitwise standardize(self(audio, offsets=offsets), ...)."""
        B = offsets.numel() - 1
        _native.check("synth_logmel_standardized", lib().synth_logmel_standardized(
            _p(audio, "audio", F32, audio.numel()), _p(offsets, "offsets", torch.int64, B + 1),
            B, 0, self.mel.data_ptr(), _p(mean, "mean", F32, MEL_FEATURES),
            _p(inv_std, "inv_std", F32, MEL_FEATURES),
            _p(rows, "rows", torch.int64, B) if rows is not None else None,
            _p(out, "features", BF16, B * MEL_FEATURES), _stream(self.device)))
        return out

    def __call__(self, audio: torch.Tensor, out: torch.Tensor | None = None,
                 offsets: torch.Tensor | None = None) -> torch.Tensor:
        """audio [B, N] (uniform) or, with offsets int64 [B + 1], a packed 1-D
        buffer of ragged voices; samples past a voice's end count as 0."""
        if offsets is None:
            B, N = audio.shape
            offp = None
        else:
            B, N = offsets.numel() - 1, 0
            offp = _p(offsets, "offsets", torch.int64, B + 1)
        if out is None:
            out = torch.empty(B, MEL_FEATURES, dtype=F32, device=self.device)
        common = (_p(audio, "audio", F32, audio.numel()), offp, B, N)
        ws = (None, 0)
        if self.method == "mfma":              # the FFT path needs no workspace
            need = lib().synth_logmel_workspace(B)
            if self._ws is None or self._ws.numel() < need:
                self._ws = torch.empty(need, dtype=torch.uint8, device=self.device)
            ws = (self._ws.data_ptr(), self._ws.numel())
        tail = (self.mel.data_ptr(), *ws, _p(out, "features", F32, B * MEL_FEATURES),
                _stream(self.device))
        if self.method == "fft":
            _native.check("synth_logmel", lib().synth_logmel(*common, *tail))
        else:
            _native.check("synth_logmel_mfma",
                          lib().synth_logmel_mfma(*common, self.dft.data_ptr(), *tail))
        return out


def colstats(x: torch.Tensor):
    rows, cols = x.shape
    s = torch.empty(cols, dtype=F32, device=x.device)
    s2 = torch.empty(cols, dtype=F32, device=x.device)
    _native.check("synth_colstats", lib().synth_colstats(
        x.data_ptr(), int(x.dtype == BF16), rows, cols, cols, s.data_ptr(), s2.data_ptr(),
        _stream(x.device)))
    return s, s2


def feature_stats(x: torch.Tensor, min_var: float = 1e-6):
    """(mean, inv_std) float32 [cols] of a float32 [rows, cols] feature matrix."""
    rows, cols = x.shape
    mean = torch.empty(cols, dtype=F32, device=x.device)
    inv_std = torch.empty(cols, dtype=F32, device=x.device)
    _native.check("synth_feature_stats", lib().synth_feature_stats(
        _p(x, "x", F32, rows * cols), rows, cols, float(min_var), mean.data_ptr(),
        inv_std.data_ptr(), _stream(x.device)))
    return mean, inv_std


def standardize(x: torch.Tensor, mean: torch.Tensor, inv_std: torch.Tensor, out=None):
    rows, cols = x.shape
    if out is None:
        out = torch.empty(rows, cols, dtype=BF16, device=x.device)
    _native.check("synth_standardize", lib().synth_standardize(
        _p(x, "x", F32), _p(mean, "mean", F32), _p(inv_std, "inv_std", F32), rows, cols,
        _p(out, "y", BF16), _stream(x.device)))
    return out


def to_bf16(x: torch.Tensor, out=None):
    if out is None:
        out = torch.empty(x.shape, dtype=BF16, device=x.device)
    _native.check("synth_to_bf16", lib().synth_to_bf16(_p(x, "x", F32), _p(out, "y", BF16),
                                                       x.numel(), _stream(x.device)))
    return out


class MLP:
    """8192 -> 1024 -> 1024 -> 78 proposal network: float32 master weights
    (transposed, K-major) with bf16 copies, Adam moments, activation buffers.
    `split_k` gives the library a workspace so that GEMMs with few output
    tiles split their reduction over workgroups."""

    def __init__(self, init: dict, device="cuda", lr=3e-4, betas=(0.9, 0.999), eps=1e-8,
                 split_k=True):
        self.device = torch.device(device)
        self.d_in, self.d_h, self.d_out = init["w1t"].shape[1], init["w1t"].shape[0], init["w3t"].shape[0]
        self.names = ("w1t", "b1", "w2t", "b2", "w3t", "b3")
        # One flat buffer per state (weights, gradients, moments): the weight
        # matrices first (their bf16 copies are one flat buffer too), then the
        # biases, so that Adam is two launches; every view starts 16-byte
        # aligned for the GEMMs' vector loads.
        mats, vecs = ("w1t", "w2t", "w3t"), ("b1", "b2", "b3")
        shapes = {k: tuple(np.asarray(init[k]).shape) for k in self.names}
        sizes = {k: int(np.prod(shapes[k])) for k in self.names}
        self._n_mat = sum(sizes[k] for k in mats)
        n_all = self._n_mat + sum(sizes[k] for k in vecs)
        flat = {s: torch.zeros(n_all, dtype=F32, device=self.device) for s in ("w", "m", "v", "g")}
        self._flat = flat
        self._wb_flat = torch.empty(self._n_mat, dtype=BF16, device=self.device)
        off, views = 0, {}
        for k in mats + vecs:
            views[k] = (off, off + sizes[k])
            off += sizes[k]
        self.w, self.m, self.v, self.g = ({k: flat[s][a:b].view(shapes[k]) for k, (a, b) in views.items()}
                                          for s in ("w", "m", "v", "g"))
        for k in self.names:
            self.w[k].copy_(torch.as_tensor(np.asarray(init[k], np.float32)))
        self.wb = {k: self._wb_flat[views[k][0]:views[k][1]].view(shapes[k]) for k in mats}
        to_bf16(flat["w"][:self._n_mat], out=self._wb_flat)
        self.lr, self.betas, self.eps = lr, betas, eps
        self.step_count = 0
        self._act_batch = 0
        self.split_k = split_k

    def _acts(self, B):
        if B != self._act_batch:
            d, h, o = self.d_in, self.d_h, self.d_out
            mk = lambda shape, dt: torch.empty(shape, dtype=dt, device=self.device)
            self.a = {"h1pre": mk((B, h), F32), "h1": mk((B, h), BF16), "h2pre": mk((B, h), F32),
                      "h2": mk((B, h), BF16), "out": mk((B, o), F32), "dz3": mk((B, o), BF16),
                      "dh2": mk((B, h), BF16), "dh1": mk((B, h), BF16),
                      "loss_rows": mk((B,), torch.float64)}
            nws = lib().synth_mlp_workspace(B, d, h, o) if self.split_k else 0
            self.ws = mk((max(nws, 1),), torch.uint8) if nws else None
            self._act_batch = B
        return self.a

    def _ws_args(self):
        return (None, 0) if self.ws is None else (self.ws.data_ptr(), self.ws.numel())

    def forward(self, x_bf16: torch.Tensor, keep=True) -> torch.Tensor:
        B = x_bf16.shape[0]
        a = self._acts(B)
        w, wb = self.w, self.wb
        _native.check("synth_mlp_forward", lib().synth_mlp_forward(
            B, self.d_in, self.d_h, self.d_out, _p(x_bf16, "x", BF16, B * self.d_in),
            wb["w1t"].data_ptr(), w["b1"].data_ptr(), wb["w2t"].data_ptr(), w["b2"].data_ptr(),
            wb["w3t"].data_ptr(), w["b3"].data_ptr(), a["h1pre"].data_ptr(), a["h1"].data_ptr(),
            a["h2pre"].data_ptr(), a["h2"].data_ptr(), a["out"].data_ptr(), *self._ws_args(),
            _stream(self.device)))
        return a["out"]

    def backward(self, x_bf16: torch.Tensor, target: torch.Tensor) -> torch.Tensor:
        """Gradients of mean((out - target)^2) into self.g; returns the loss (0-d, float64)."""
        B = x_bf16.shape[0]
        a, wb, g = self.a, self.wb, self.g
        _native.check("synth_mlp_backward", lib().synth_mlp_backward(
            B, self.d_in, self.d_h, self.d_out, x_bf16.data_ptr(), wb["w2t"].data_ptr(),
            wb["w3t"].data_ptr(), a["h1pre"].data_ptr(), a["h1"].data_ptr(), a["h2pre"].data_ptr(),
            a["h2"].data_ptr(), a["out"].data_ptr(), _p(target, "target", F32, B * self.d_out),
            g["w1t"].data_ptr(), g["b1"].data_ptr(), g["w2t"].data_ptr(), g["b2"].data_ptr(),
            g["w3t"].data_ptr(), g["b3"].data_ptr(), a["dz3"].data_ptr(), a["dh2"].data_ptr(),
            a["dh1"].data_ptr(), a["loss_rows"].data_ptr(), *self._ws_args(), _stream(self.device)))
        return sum_f64(a["loss_rows"][:B], 1.0 / (B * self.d_out))

    def adam_step(self):
        """One Adam step on every parameter: the weight matrices (refreshing
        their bf16 copies) and the biases, two launches over the flat buffers."""
        self.step_count += 1
        b1, b2 = self.betas
        f, n = self._flat, self._n_mat
        for a, b, wb in ((0, n, self._wb_flat), (n, f["w"].numel(), None)):
            _native.check("synth_adam", lib().synth_adam(
                b - a, f["w"][a:].data_ptr(), wb.data_ptr() if wb is not None else None,
                f["g"][a:].data_ptr(), f["m"][a:].data_ptr(), f["v"][a:].data_ptr(),
                float(self.lr), float(b1), float(b2), float(self.eps), self.step_count,
                _stream(self.device)))

    def train_step(self, x_bf16, target):
        self.forward(x_bf16)
        loss = self.backward(x_bf16, target)
        self.adam_step()
        return loss

    def state_dict(self):
        return {"w": {k: v.detach().cpu().clone() for k, v in self.w.items()},
                "m": {k: v.detach().cpu().clone() for k, v in self.m.items()},
                "v": {k: v.detach().cpu().clone() for k, v in self.v.items()},
                "step": self.step_count}

    def load_state_dict(self, sd):
        for k in self.names:
            self.w[k].copy_(sd["w"][k])
            self.m[k].copy_(sd["m"][k])
            self.v[k].copy_(sd["v"][k])
        for k in self.wb:
            to_bf16(self.w[k], out=self.wb[k])
        self.step_count = int(sd["step"])


def logit_init(u: torch.Tensor, eps: float = 1e-4):
    """(z, u') with z = logit(clamp(u, eps, 1 - eps)) and u' = sigmoid(z)."""
    z = torch.empty_like(u)
    u2 = torch.empty_like(u)
    _native.check("synth_logit_init", lib().synth_logit_init(
        _p(u, "u", F32), _p(z, "z", F32), _p(u2, "u_out", F32), u.numel(), float(eps),
        _stream(u.device)))
    return z, u2


def logit_adam(z, u, grad_u, m, v, step, lr=0.05, betas=(0.9, 0.999), eps=1e-8):
    """In place: Adam on z with dL/dz = grad_u u (1 - u); u <- sigmoid(z)."""
    n = z.numel()
    _native.check("synth_logit_adam", lib().synth_logit_adam(
        n, _p(z, "z", F32, n), _p(u, "u", F32, n), _p(grad_u, "grad_u", F32, n),
        _p(m, "m", F32, n), _p(v, "v", F32, n), float(lr), float(betas[0]), float(betas[1]),
        float(eps), int(step), _stream(z.device)))


def best_update(loss, rows, cols, row_stride, col_stride, best, best_idx=None, col_base=0,
                params=None, best_params=None):
    """Per-row running minimum of loss (see synth_best_update in synth.h)."""
    pd = 0 if params is None else best_params.shape[-1]
    _native.check("synth_best_update", lib().synth_best_update(
        _p(loss, "loss", torch.float64), rows, cols, row_stride, col_stride, col_base,
        _p(params, "params", F32) if params is not None else None, pd,
        _p(best, "best", torch.float64, rows),
        _p(best_idx, "best_idx", torch.int64, rows) if best_idx is not None else None,
        _p(best_params, "best_params", F32, rows * pd) if best_params is not None else None,
        _stream(loss.device)))


# ---------------------------------------------------------------------------
# Training the proposal on rendered voices
# ---------------------------------------------------------------------------
TRAIN_BLOCK, TEST_BLOCK = 9 * 1024, 1024


def train_ids(first: int, count: int, device="cuda") -> torch.Tensor:
    """Global voice indices of training voices first .. first + count - 1,
    counted in the corpus order with every test block of 1024 skipped (the
    split of Section 2.1: 9 x 1024 train voices, then 1024 test voices)."""
    i = torch.arange(first, first + count, device=device, dtype=torch.int64)
    return (i // TRAIN_BLOCK) * (TRAIN_BLOCK + TEST_BLOCK) + i % TRAIN_BLOCK


_LENGTHS = {}


def _lengths_tensor(lengths_s, sample_rate, device) -> torch.Tensor:
    """Voice lengths in samples (int64, on `device`), made once per (lengths,
    rate, device): building a device tensor from a host list is a blocking
    copy from pageable memory, which waits for the work queued on every
    stream and so would stall a loop that overlaps streams."""
    key = (tuple(float(x) for x in lengths_s), float(sample_rate), str(device))
    t = _LENGTHS.get(key)
    if t is None:
        t = torch.tensor([int(round(x * sample_rate)) for x in lengths_s], dtype=torch.int64,
                         device=device)
        _LENGTHS[key] = t
    return t


def ragged_offsets(ids: torch.Tensor, lengths_s=(1, 2, 3, 4), sample_rate=44100.0) -> torch.Tensor:
    """offsets [B + 1] of voices rendered lengths_s[g mod len] seconds long."""
    per = _lengths_tensor(lengths_s, sample_rate, ids.device)
    n = per[ids % len(lengths_s)]
    return torch.cat([torch.zeros(1, dtype=torch.int64, device=ids.device), torch.cumsum(n, 0)])


class Proposal:
    """Audio -> parameter estimate: log-mel features, standardised with fixed
    statistics, through the MLP; returns u in (0, 1), float32 [B, 78]."""

    def __init__(self, mlp: MLP, logmel: LogMel, mean: torch.Tensor, inv_std: torch.Tensor):
        self.mlp, self.logmel, self.mean, self.inv_std = mlp, logmel, mean, inv_std

    def features(self, audio, offsets=None):
        return standardize(self.logmel(audio, offsets=offsets), self.mean, self.inv_std)

    def __call__(self, audio, offsets=None):
        return self.mlp.forward(self.features(audio, offsets)).clone()


_TUNER = None


def render_batch(seed, ids, nebula_table, lengths_s=(1, 2, 3, 4), tune: bool = True,
                 return_ids: bool = False):
    """(u, packed audio, offsets) of voices ids drawn and rendered on the GPU
    (with the launch plan the autotuner picked for this batch shape).  The
    voices come back ordered longest first; u and the audio stay aligned
    (return_ids=True appends the voice ids in that order)."""
    global _TUNER
    from . import synth_render, synth_sample_params
    # longest voices first: workgroups are dispatched in voice order, so the
    # long voices start early and the short ones fill the tail of the launch
    per = _lengths_tensor(lengths_s, 44100.0, ids.device)
    ids = ids[torch.argsort(-per[ids % len(lengths_s)], stable=True)]
    offs = ragged_offsets(ids, lengths_s)
    u = synth_sample_params(seed, voice_ids=ids)
    if tune:
        if _TUNER is None:
            from .autotune import RenderTuner, default_candidates
            # Every step renders new voices (new note lengths and silent tails):
            # persistent round-robin grids, whose speed depends on the order of
            # the voices' costs, are left out; slices balance the load per voice.
            cands = [p for p in default_candidates(ids.numel(), False) if not p[2]]
            _TUNER = RenderTuner(reps=3, candidates=cands)
        # every batch of B consecutive training voices has the same length mix
        # when B is a multiple of the cycle, so the shape is named, not read back
        B, c = ids.numel(), len(lengths_s)
        key, out = None, None
        if B % c == 0:
            key = f"train:{B}:{tuple(lengths_s)}"
            total = (B // c) * sum(int(round(x * 44100.0)) for x in lengths_s)
            out = torch.empty(total, dtype=F32, device=ids.device)
        lmax = max(int(round(x * 44100.0)) for x in lengths_s)
        audio = _TUNER.render(u, nebula_table, offsets=offs, voice_ids=ids, noise_seed=seed,
                              key=key, out=out, max_samples=lmax)
    else:
        audio = synth_render(u, nebula_table, offsets=offs, voice_ids=ids, noise_seed=seed)
    if return_ids:
        return u, audio, offs, ids
    return u, audio, offs


def train_pipelined(net: "MLP", lm: LogMel, nebula_table, mean, inv_std, steps: int,
                    batch: int, seed: int, lengths_s=(1, 2, 3, 4), lr_at=None, first: int = 1,
                    on_step=None, group: int = 2, tune: bool = True):
    """Training steps 0 .. steps - 1 on the voices of batches first, first + 1,
    ...  The voices of `group` consecutive steps are drawn, rendered (one
    launch: the short voices of one step fill the tail the long ones leave)
    and featurised together (a last, partial group too: its extra voices are
    rendered and not trained on), then split back into their steps in the
    order a per-step render gives them; while the MLP takes the steps of one
    group on a second stream, the next group is rendered on the caller's
    stream (two feature buffers, events between the streams), so the
    VALU-bound render overlaps the matrix-core GEMMs.  With one launch plan's runs per segment
    (tune=False, or when the autotuner picks the same for both batch shapes)
    every step computes bitwise what it computes when the steps run one after
    another.  lr_at(s) gives the learning rate of step s; on_step(s, losses)
    is called after step s is enqueued; the losses are written on the second
    stream, so it must synchronise the device before reading one (the
    caller's stream waits for the second one when this returns).  Returns the
    per-step losses (0-d float64 tensors)."""
    main = torch.cuda.current_stream()
    side = torch.cuda.Stream()
    G = max(1, int(group))
    per = _lengths_tensor(lengths_s, 44100.0, torch.device("cuda"))
    xb = [torch.empty(G * batch, MEL_FEATURES, dtype=BF16, device="cuda") for _ in range(2)]
    ready = [torch.cuda.Event(), torch.cuda.Event()]
    done = [torch.cuda.Event(), torch.cuda.Event()]
    us = [None, None]
    losses = []
    ngroups = (steps + G - 1) // G

    def prepare(k, slot):
        # always G steps' voices (a last, partial group renders voices it does
        # not train on), so that every launch has the one tuned batch shape
        n = G
        ids = torch.cat([train_ids((first + k * G + g) * batch, batch) for g in range(n)])
        u, audio, offs = render_batch(seed, ids, nebula_table, lengths_s, tune=tune)
        # render_batch orders the voices longest first (stable); the rows of
        # step g, in that order, are where the sorted positions fall in
        # [g batch, (g + 1) batch): gather them step by step
        order = torch.argsort(-per[ids % len(lengths_s)], stable=True)
        rows = torch.argsort(order // batch, stable=True)
        # features standardised in the log-mel kernel, each voice's row
        # written straight to its place in the steps' order
        lm.standardized(audio, offs, mean, inv_std, out=xb[slot], rows=torch.argsort(rows))
        us[slot] = u.index_select(0, rows)
        ready[slot].record(main)

    if steps <= 0:
        return losses
    prepare(0, 0)
    for k in range(ngroups):
        c = k % 2
        n = min(G, steps - k * G)
        with torch.cuda.stream(side):
            side.wait_event(ready[c])
            for g in range(n):
                s = k * G + g
                if lr_at is not None:
                    net.lr = lr_at(s)
                rows = slice(g * batch, (g + 1) * batch)
                losses.append(net.train_step(xb[c][rows], us[c][rows]).clone())
            done[c].record(side)
        us[c].record_stream(side)        # drawn on the main stream, read on the side stream
        if k + 1 < ngroups:
            if k >= 1:
                main.wait_event(done[1 - c])   # group k - 1 is done with its buffers
            prepare(k + 1, 1 - c)
        if on_step is not None:
            for g in range(n):
                on_step(k * G + g, losses)
    main.wait_stream(side)
    return losses


def train_proposal(nebula_table, steps: int, init, batch: int = 4096, seed: int = 10,
                   lengths_s=(1, 2, 3, 4), lr: float = 3e-4, warmup: int = 500,
                   log_every: int = 0, log=print):
    """Train the proposal on freshly rendered training voices: each step draws
    `batch` new voices, renders them (ragged lengths), computes log-mel
    features and takes one Adam step on the MSE between the MLP's sigmoid
    output and the drawn u (render and MLP of consecutive steps overlapped,
    train_pipelined).  `init`: the initial weights (dict of float32 arrays,
    as MLP takes them).  Feature statistics come from the first batch.
    Returns (Proposal, history of (step, loss))."""
    lm = LogMel()
    net = MLP(init, lr=lr)
    _, audio, offs = render_batch(seed, train_ids(0, batch), nebula_table, lengths_s)
    mean, inv_std = feature_stats(lm(audio, offsets=offs))
    del audio
    hist = []

    def on_step(s, losses):
        if log_every and ((s + 1) % log_every == 0 or s + 1 == steps):
            torch.cuda.synchronize()       # the losses are written on the MLP's stream
            hist.extend((i, float(losses[i])) for i in range(len(hist), s + 1))
            log(f"train step {s + 1}/{steps} loss {hist[-1][1]:.5f}")

    losses = train_pipelined(net, lm, nebula_table, mean, inv_std, steps, batch, seed, lengths_s,
                             lr_at=lambda s: lr * min(1.0, (s + 1) / max(1, warmup)),
                             on_step=on_step)
    hist.extend((i, float(losses[i])) for i in range(len(hist), len(losses)))
    return Proposal(net, lm, mean, inv_std), hist


def heldout_mse(proposal: Proposal, nebula_table, seed: int = 11, count: int = 4096,
                lengths_s=(1, 2, 3, 4), batch: int = 1024, per_param: bool = False):
    """Mean squared error of the proposal's u on held-out voices (another
    seed); per_param=True returns the float64 [78] per-parameter errors."""
    per = torch.zeros(78, dtype=torch.float64, device="cuda")
    for first in range(0, count, batch):
        ids = torch.arange(first, min(first + batch, count), device="cuda", dtype=torch.int64)
        u, audio, offs = render_batch(seed, ids, nebula_table, lengths_s)
        est = proposal(audio, offs)
        diff_reduce(est, u, kind=1, axis=0, scale=1.0 / count, out=per, accumulate=True)
    if per_param:
        return per.cpu()
    return float(sum_f64(per, 1.0 / 78))


def heldout_logmel_l1(proposal: Proposal, nebula_table, seed: int = 11, count: int = 4096,
                      lengths_s=(1, 2, 3, 4), batch: int = 1024) -> float:
    """Re-rendered log-mel L1 of the proposal on held-out voices: each voice
    (another seed, lengths 1-4 s) is re-rendered from the proposal's u with
    its own voice id and noise key, and the mean |log-mel difference| over
    the 128 x 64 features is averaged over the voices."""
    tot = torch.zeros((), dtype=torch.float64, device="cuda")
    lm = proposal.logmel
    for first in range(0, count, batch):
        ids = torch.arange(first, min(first + batch, count), device="cuda", dtype=torch.int64)
        u, audio, offs, ids = render_batch(seed, ids, nebula_table, lengths_s, return_ids=True)
        est = proposal(audio, offs)
        from . import synth_render
        again = synth_render(est.contiguous(), nebula_table, offsets=offs, voice_ids=ids,
                             noise_seed=seed)
        fa, fb = lm(again, offsets=offs), lm(audio, offsets=offs)
        d = diff_reduce(fa, fb, kind=0, axis=1, scale=1.0 / (fa.shape[1] * count))
        tot += sum_f64(d)
    return float(tot)
