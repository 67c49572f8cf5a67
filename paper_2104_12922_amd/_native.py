"""ctypes binding of libsynth.so (include/synth.h).  Argument marshalling only:
every step of the render runs in the library's HIP kernels."""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libsynth.so")

SYNTH_OK = 0
NUM_PARAMS = 78


class SynthError(RuntimeError):
    def __init__(self, fn: str, status: int, msg: str):
        super().__init__(f"{fn} failed: {msg} (status {status})")
        self.status = status


class SynthConfig(ctypes.Structure):
    _fields_ = [("sample_rate", ctypes.c_double),
                ("control_rate", ctypes.c_double),
                ("noise_seed", ctypes.c_uint64),
                ("mix_mode", ctypes.c_int32),
                ("reserved", ctypes.c_int32),
                ("nebula", ctypes.POINTER(ctypes.c_double))]


_lib = None


def lib() -> ctypes.CDLL:
    """Load libsynth.so (fails loudly if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2104_12922_amd.build`")
        L = ctypes.CDLL(LIB_PATH)
        L.synth_num_params.restype = ctypes.c_int
        L.synth_status_string.restype = ctypes.c_char_p
        L.synth_num_params.argtypes = []
        L.synth_param_info.restype = ctypes.c_int
        L.synth_param_info.argtypes = [ctypes.c_int, ctypes.POINTER(ctypes.c_char_p)] + \
            [ctypes.POINTER(ctypes.c_double)] * 3 + [ctypes.POINTER(ctypes.c_int)]
        L.synth_status_string.argtypes = [ctypes.c_int]
        L.synth_is_test.restype = ctypes.c_int
        L.synth_is_test.argtypes = [ctypes.c_uint64]
        L.synth_sample_params.restype = ctypes.c_int
        L.synth_sample_params.argtypes = [ctypes.c_uint64, ctypes.c_uint64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p]
        render_args = [ctypes.POINTER(SynthConfig), ctypes.c_void_p, ctypes.c_void_p,
                       ctypes.c_uint64, ctypes.c_int64, ctypes.c_void_p, ctypes.c_int64,
                       ctypes.c_void_p]
        L.synth_render.restype = ctypes.c_int
        L.synth_render.argtypes = render_args + [ctypes.c_void_p]
        L.synth_render_noalloc.restype = ctypes.c_int
        L.synth_render_noalloc.argtypes = render_args + [ctypes.c_void_p]
        L.synth_generate.restype = ctypes.c_int
        L.synth_generate.argtypes = [ctypes.POINTER(SynthConfig), ctypes.c_uint64, ctypes.c_void_p,
                                     ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64,
                                     ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p,
                                     ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.synth_render_workspace.restype = ctypes.c_size_t
        L.synth_render_workspace.argtypes = [ctypes.POINTER(SynthConfig), ctypes.c_int64,
                                             ctypes.c_int64]
        L.synth_render_ws.restype = ctypes.c_int
        L.synth_render_ws.argtypes = render_args + [ctypes.c_void_p, ctypes.c_size_t,
                                                    ctypes.c_void_p]
        L.synth_render_plan.restype = ctypes.c_int
        L.synth_render_plan.argtypes = render_args + [ctypes.c_int] * 4 + [ctypes.c_void_p]
        L.synth_render_plan_workspace.restype = ctypes.c_size_t
        L.synth_render_plan_workspace.argtypes = [ctypes.POINTER(SynthConfig), ctypes.c_int64,
                                                  ctypes.c_int64]
        L.synth_render_plan_ws.restype = ctypes.c_int
        L.synth_render_plan_ws.argtypes = (render_args[:7] + [ctypes.c_int64] + render_args[7:] +
                                           [ctypes.c_int] * 4 +
                                           [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                            ctypes.c_void_p])
        L.synth_mrstft_loss.restype = ctypes.c_int
        L.synth_mrstft_loss.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_int64,
                                        ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                        ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.synth_mrstft_target_bytes.restype = ctypes.c_size_t
        L.synth_mrstft_target_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64]
        L.synth_mrstft_target.restype = ctypes.c_int
        L.synth_mrstft_target.argtypes = [ctypes.c_void_p, ctypes.c_int64, ctypes.c_int64,
                                          ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        L.synth_mrstft_loss_cached.restype = ctypes.c_int
        L.synth_mrstft_loss_cached.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p,
                                               ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t,
                                               ctypes.c_void_p]
        L.synth_mrstft_workspace.restype = ctypes.c_size_t
        L.synth_mrstft_workspace.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int]
        L.synth_render_backward_workspace.restype = ctypes.c_size_t
        L.synth_render_backward_workspace.argtypes = [ctypes.POINTER(SynthConfig), ctypes.c_int64,
                                                      ctypes.c_int64]
        L.synth_render_backward.restype = ctypes.c_int
        L.synth_render_backward.argtypes = [ctypes.POINTER(SynthConfig), ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_uint64, ctypes.c_int64,
                                            ctypes.c_int64, ctypes.c_void_p, ctypes.c_void_p,
                                            ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p]
        _lib = L
    return _lib


def status_string(st: int) -> str:
    return lib().synth_status_string(st).decode()


def check(fn: str, st: int) -> None:
    if st != SYNTH_OK:
        raise SynthError(fn, st, status_string(st))


def make_config(nebula_table, sample_rate=44100.0, control_rate=441.0, noise_seed=0,
                mix_mode=0):
    """Returns (config, keepalive): the nebula array must outlive the call."""
    tab = np.ascontiguousarray(np.asarray(nebula_table, dtype=np.float64).reshape(NUM_PARAMS, 4))
    cfg = SynthConfig(float(sample_rate), float(control_rate), int(noise_seed) & (2**64 - 1),
                      int(mix_mode), 0, tab.ctypes.data_as(ctypes.POINTER(ctypes.c_double)))
    return cfg, tab
