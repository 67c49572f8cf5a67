"""MI355X-native batched modular-synth voice renderer (arXiv 2104.12922).

Python face of libsynth.so: the functions below take torch tensors that live on
the GPU, pass their device pointers and the current HIP stream to the C ABI
(include/synth.h), and return tensors.  PyTorch provides device memory and
streams only; the parameter draw and every stage of the render run in the
library's HIP kernels.  There is no CPU fallback: without the built library or
a GPU these functions raise.
"""
from __future__ import annotations

import numpy as np
import torch

from . import _native

NUM_PARAMS = _native.NUM_PARAMS

__all__ = ["synth_sample_params", "synth_render", "synth_render_plan", "synth_is_test",
           "synth_mrstft_loss", "synth_mrstft_target", "MrstftTarget",
           "synth_render_backward", "SynthRender", "MRSTFTLoss",
           "NUM_PARAMS", "SynthError"]

SynthError = _native.SynthError


def _stream(device) -> int:
    return torch.cuda.current_stream(device).cuda_stream


def _dev_ptr(t, name, dtype, numel=None):
    if t is None:
        return None
    if not isinstance(t, torch.Tensor) or not t.is_cuda:
        raise TypeError(f"{name} must be a CUDA (HIP) tensor")
    if dtype == torch.uint64 and t.dtype == torch.int64:
        dtype = torch.int64          # voice ids: same 64-bit pattern
    if t.dtype != dtype or not t.is_contiguous():
        raise TypeError(f"{name} must be a contiguous {dtype} tensor")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")
    return t.data_ptr()


def synth_param_info(p: int) -> dict:
    """Name and default nebula range of parameter p (see synth.h)."""
    import ctypes
    nm = ctypes.c_char_p()
    lo, hi, cv = ctypes.c_double(), ctypes.c_double(), ctypes.c_double()
    sym = ctypes.c_int()
    _native.check("synth_param_info", _native.lib().synth_param_info(
        int(p), ctypes.byref(nm), ctypes.byref(lo), ctypes.byref(hi), ctypes.byref(cv),
        ctypes.byref(sym)))
    return {"name": nm.value.decode(), "min": lo.value, "max": hi.value, "curve": cv.value,
            "symmetric": bool(sym.value)}


def synth_is_test(g: int) -> bool:
    return bool(_native.lib().synth_is_test(int(g)))


def synth_sample_params(seed: int, first_g: int = 0, batch: int | None = None,
                        voice_ids: torch.Tensor | None = None, out: torch.Tensor | None = None,
                        device="cuda") -> torch.Tensor:
    """Normalised parameters [B, 78] float32 drawn from Philox4x32-10 (see synth.h)."""
    if voice_ids is not None:
        batch = voice_ids.numel()
        device = voice_ids.device
    if batch is None:
        raise ValueError("batch or voice_ids is required")
    if out is None:
        out = torch.empty(batch, NUM_PARAMS, dtype=torch.float32, device=device)
    ids = _dev_ptr(voice_ids, "voice_ids", torch.uint64, batch) if voice_ids is not None else None
    _native.check("synth_sample_params", _native.lib().synth_sample_params(
        int(seed) & (2**64 - 1), int(first_g), int(batch), ids,
        _dev_ptr(out, "out", torch.float32, batch * NUM_PARAMS), _stream(out.device)))
    return out


def _render_common(params, nebula, n_samples, offsets, voice_ids, first_g, noise_seed, mix_mode,
                   sample_rate, control_rate, out):
    B = params.shape[0]
    cfg, keep = _native.make_config(nebula, sample_rate, control_rate, noise_seed, mix_mode)
    if offsets is not None:
        total = int(offsets[-1].item()) if out is None else out.numel()
    else:
        total = B * int(n_samples)
    if out is None:
        out = torch.empty(total, dtype=torch.float32, device=params.device)
    args = (cfg, _dev_ptr(params, "params", torch.float32, B * NUM_PARAMS),
            _dev_ptr(voice_ids, "voice_ids", torch.uint64, B) if voice_ids is not None else None,
            int(first_g), int(B),
            _dev_ptr(offsets, "offsets", torch.int64, B + 1) if offsets is not None else None,
            int(n_samples) if offsets is None else 0,
            _dev_ptr(out, "audio", torch.float32, total))
    return args, out, keep


def synth_render(params: torch.Tensor, nebula, n_samples: int | None = None,
                 offsets: torch.Tensor | None = None, voice_ids: torch.Tensor | None = None,
                 first_g: int = 0, noise_seed: int = 0, mix_mode: int = 0,
                 sample_rate: float = 44100.0, control_rate: float = 441.0,
                 out: torch.Tensor | None = None) -> torch.Tensor:
    """Render B voices.  Uniform: returns [B, n_samples]; ragged (offsets given):
    returns the packed 1-D buffer of offsets[-1] samples.  Small uniform
    batches get a workspace for the chunk-start carries (`synth_render_ws`)."""
    args, out, keep = _render_common(params, nebula, n_samples, offsets, voice_ids, first_g,
                                     noise_seed, mix_mode, sample_rate, control_rate, out)
    L = _native.lib()
    need = 0 if offsets is not None else L.synth_render_workspace(
        ctypes_ref(args[0]), params.shape[0], int(n_samples))
    if need:
        ws = torch.empty(need, dtype=torch.uint8, device=params.device)
        st = L.synth_render_ws(ctypes_ref(args[0]), *args[1:], ws.data_ptr(), ws.numel(),
                               _stream(params.device))
        _native.check("synth_render_ws", st)
    else:
        st = L.synth_render(ctypes_ref(args[0]), *args[1:], _stream(params.device))
        _native.check("synth_render", st)
    del keep
    if offsets is None:
        return out.view(params.shape[0], int(n_samples))
    return out


def synth_render_plan(params: torch.Tensor, nebula, runs_per_segment: int, slices_per_voice: int,
                      persistent: bool = False, grid_blocks: int = 0, n_samples: int | None = None,
                      offsets: torch.Tensor | None = None, voice_ids: torch.Tensor | None = None,
                      first_g: int = 0, noise_seed: int = 0, mix_mode: int = 0,
                      sample_rate: float = 44100.0, control_rate: float = 441.0,
                      out: torch.Tensor | None = None, carries: bool = True,
                      max_samples: int | None = None, workspace: torch.Tensor | None = None,
                      order: torch.Tensor | None = None) -> torch.Tensor:
    """Render with an explicit launch plan.  With slices_per_voice > 1 and
    `carries`, the chunk-start phase carries are computed first in a
    workspace (`synth_render_plan_ws`); `max_samples` (longest voice, ragged
    batches) avoids reading the offsets back; `workspace` may be given to
    reuse a buffer.  `order` (int32 [B], a permutation) is the order in which
    workgroups take the voices (the output does not depend on it)."""
    args, out, keep = _render_common(params, nebula, n_samples, offsets, voice_ids, first_g,
                                     noise_seed, mix_mode, sample_rate, control_rate, out)
    L = _native.lib()
    plan = (int(runs_per_segment), int(slices_per_voice), int(bool(persistent)), int(grid_blocks))
    B = params.shape[0]
    use_carries = carries and slices_per_voice > 1 and B > 0
    if use_carries or order is not None:
        ordp = _dev_ptr(order, "order", torch.int32, B) if order is not None else None
        lmax, wsp, wsn = 0, None, 0
        if use_carries:
            if offsets is None:
                lmax = int(n_samples)
            elif max_samples is not None:
                lmax = int(max_samples)
            else:
                lmax = int(torch.diff(offsets).max().item())
            need = L.synth_render_plan_workspace(ctypes_ref(args[0]), B, max(lmax, 1))
            if workspace is None or workspace.numel() < need:
                workspace = torch.empty(max(need, 1), dtype=torch.uint8, device=params.device)
            wsp, wsn = workspace.data_ptr(), workspace.numel()
        st = L.synth_render_plan_ws(ctypes_ref(args[0]), *args[1:7], lmax, args[7], *plan, ordp,
                                    wsp, wsn, _stream(params.device))
        _native.check("synth_render_plan_ws", st)
    else:
        st = L.synth_render_plan(ctypes_ref(args[0]), *args[1:], *plan, _stream(params.device))
        _native.check("synth_render_plan", st)
    del keep
    if offsets is None:
        return out.view(params.shape[0], int(n_samples))
    return out


def synth_mrstft_workspace(batch: int, n_samples: int, grad: bool = False) -> torch.Tensor:
    """A device workspace large enough for synth_mrstft_loss."""
    need = _native.lib().synth_mrstft_workspace(int(batch), int(n_samples), int(bool(grad)))
    if need == 0:
        raise ValueError("invalid MR-STFT sizes")
    return torch.empty(need, dtype=torch.uint8, device="cuda")


class MrstftTarget:
    """Log-magnitude spectra of a fixed [B, N] target, computed once by
    synth_mrstft_target and reused by synth_mrstft_loss(x, <this>)."""

    def __init__(self, target: torch.Tensor):
        if target.dim() != 2:
            raise ValueError("target must be [B, N]")
        B, N = target.shape
        self.shape = target.shape
        self.device = target.device
        nbytes = _native.lib().synth_mrstft_target_bytes(int(B), int(N))
        self.tlog = torch.empty(max(nbytes, 8) // 4 + 1, dtype=torch.float32,
                                device=target.device)
        _native.check("synth_mrstft_target", _native.lib().synth_mrstft_target(
            _dev_ptr(target, "target", torch.float32, B * N), B, N, self.tlog.data_ptr(),
            self.tlog.numel() * 4, _stream(target.device)))


def synth_mrstft_target(target: torch.Tensor) -> MrstftTarget:
    return MrstftTarget(target)


def synth_mrstft_loss(x: torch.Tensor, target, grad: bool = False,
                      workspace: torch.Tensor | None = None, out_grad: torch.Tensor | None = None):
    """Per-voice multi-resolution log-magnitude STFT L1 (float64 [B]) and, if
    grad, d loss[b] / d x[b] (float32 [B, N]) - see synth.h.  target is a
    [B, N] float32 tensor or an MrstftTarget of one (spectra computed once)."""
    cached = isinstance(target, MrstftTarget)
    if x.shape != target.shape or x.dim() != 2:
        raise ValueError("x and target must both be [B, N]")
    B, N = x.shape
    loss = torch.empty(B, dtype=torch.float64, device=x.device)
    g = (out_grad if out_grad is not None else torch.empty_like(x)) if grad else None
    need = _native.lib().synth_mrstft_workspace(int(B), int(N), int(bool(grad)))
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=x.device)
    if cached:
        fn = "synth_mrstft_loss_cached"
        tptr = (target.tlog.data_ptr(), target.tlog.numel() * 4)
    else:
        fn, tptr = "synth_mrstft_loss", (_dev_ptr(target, "target", torch.float32, B * N),)
    _native.check(fn, getattr(_native.lib(), fn)(
        _dev_ptr(x, "x", torch.float32, B * N), *tptr,
        B, N, _dev_ptr(loss, "loss", torch.float64, B),
        _dev_ptr(g, "grad", torch.float32, B * N) if grad else None, workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), _stream(x.device)))
    return (loss, g) if grad else loss


def synth_render_backward(params: torch.Tensor, grad_audio: torch.Tensor, nebula,
                          voice_ids: torch.Tensor | None = None, first_g: int = 0,
                          noise_seed: int = 0, sample_rate: float = 44100.0,
                          control_rate: float = 441.0, workspace: torch.Tensor | None = None,
                          out: torch.Tensor | None = None) -> torch.Tensor:
    """d(sum grad_audio * render(params)) / d params, float32 [B, 78] (see synth.h)."""
    import ctypes
    B, N = grad_audio.shape
    cfg, keep = _native.make_config(nebula, sample_rate, control_rate, noise_seed, 0)
    L = _native.lib()
    need = L.synth_render_backward_workspace(ctypes.byref(cfg), B, N)
    if workspace is None or workspace.numel() * workspace.element_size() < need:
        workspace = torch.empty(max(need, 8), dtype=torch.uint8, device=params.device)
    gp = out if out is not None else torch.empty(B, NUM_PARAMS, dtype=torch.float32,
                                                 device=params.device)
    _native.check("synth_render_backward", L.synth_render_backward(
        ctypes.byref(cfg), _dev_ptr(params, "params", torch.float32, B * NUM_PARAMS),
        _dev_ptr(voice_ids, "voice_ids", torch.uint64, B) if voice_ids is not None else None,
        int(first_g), B, N, _dev_ptr(grad_audio, "grad_audio", torch.float32, B * N),
        _dev_ptr(gp, "grad_params", torch.float32, B * NUM_PARAMS), workspace.data_ptr(),
        workspace.numel() * workspace.element_size(), _stream(params.device)))
    del keep
    return gp


def synth_render_backward_workspace(nebula, batch: int, n_samples: int,
                                    sample_rate: float = 44100.0,
                                    control_rate: float = 441.0) -> torch.Tensor:
    """A device workspace large enough for synth_render_backward."""
    import ctypes
    cfg, keep = _native.make_config(nebula, sample_rate, control_rate, 0, 0)
    need = _native.lib().synth_render_backward_workspace(ctypes.byref(cfg), batch, n_samples)
    del keep
    if need == 0:
        raise ValueError("invalid configuration for synth_render_backward")
    return torch.empty(need, dtype=torch.uint8, device="cuda")


class SynthRender(torch.autograd.Function):
    """Differentiable render of uniform-length voices: forward = synth_render,
    backward = synth_render_backward (envelopes and oscillators are recomputed;
    only the parameters are saved)."""

    @staticmethod
    def forward(ctx, params, nebula, n_samples, first_g=0, noise_seed=0, sample_rate=44100.0,
                control_rate=441.0):
        p = params.detach().contiguous()
        y = synth_render(p, nebula, n_samples=n_samples, first_g=first_g, noise_seed=noise_seed,
                         sample_rate=sample_rate, control_rate=control_rate)
        ctx.save_for_backward(p)
        ctx.cfg = (nebula, first_g, noise_seed, sample_rate, control_rate)
        return y

    @staticmethod
    def backward(ctx, gy):
        (p,) = ctx.saved_tensors
        nebula, first_g, noise_seed, sr, rc = ctx.cfg
        gp = synth_render_backward(p, gy.contiguous().float(), nebula, first_g=first_g,
                                   noise_seed=noise_seed, sample_rate=sr, control_rate=rc)
        return gp, None, None, None, None, None, None


class MRSTFTLoss(torch.autograd.Function):
    """Per-voice multi-resolution log-magnitude STFT L1 (float64 [B]) with its
    gradient w.r.t. the render computed by the same kernel."""

    @staticmethod
    def forward(ctx, x, target):
        loss, g = synth_mrstft_loss(x.detach().contiguous(), target.contiguous(), grad=True)
        ctx.save_for_backward(g)
        return loss

    @staticmethod
    def backward(ctx, gl):
        (g,) = ctx.saved_tensors
        from .learned import scale_rows
        return scale_rows(g, gl.detach().to(torch.float64).contiguous()), None


def ctypes_ref(cfg):
    import ctypes
    return ctypes.byref(cfg)
