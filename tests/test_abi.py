"""C-ABI tests that need no GPU: the library loads, exports every symbol the
header declares, and rejects bad arguments on the host before any launch."""
import ctypes
import os
import re

import numpy as np
import pytest

import workloads as W
from paper_2104_12922_amd import _native

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
EINVAL, EUNSUP = -1, -4


def header_functions():
    names = []
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if h.endswith(".h"):
            txt = open(os.path.join(ROOT, "include", h)).read()
            txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
            names += re.findall(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_\s\*]*?\b(synth_[a-z0-9_]+)\s*\(",
                                txt, flags=re.M)
    return sorted(set(names))


def test_library_exports_every_declared_symbol():
    L = _native.lib()
    names = header_functions()
    assert "synth_render" in names and "synth_sample_params" in names
    for n in names:
        assert hasattr(L, n), f"libsynth.so does not export {n}"


def test_scalar_entry_points():
    L = _native.lib()
    assert L.synth_num_params() == 78 == len(W.param_names())
    assert _native.status_string(0) == "ok"
    for g in (0, 9215, 9216, 10239, 10240, 19455, 19456, 2**40 + 9 * 1024):
        assert bool(L.synth_is_test(g)) == ((g // 1024) % 10 == 9)


def test_param_info_matches_default_nebula():
    import paper_2104_12922_amd as S
    names = W.param_names()
    tab = W.default_nebula().table()
    for p in range(78):
        info = S.synth_param_info(p)
        assert info["name"] == names[p]
        assert (info["min"], info["max"], info["curve"], float(info["symmetric"])) == tuple(tab[p])
    L = _native.lib()
    assert L.synth_param_info(78, None, None, None, None, None) == EINVAL
    assert L.synth_param_info(-1, None, None, None, None, None) == EINVAL


def _render(cfg, params=1, ids=None, B=1, offsets=None, n=1000, audio=1, rps=4, slices=1,
            persistent=0, grid=0):
    L = _native.lib()
    ref = ctypes.byref(cfg) if cfg is not None else None
    return L.synth_render_plan(ref, params, ids, 0, B, offsets, n, audio, rps, slices,
                               persistent, grid, None)


def cfg_with(**kw):
    tab = W.default_nebula().table()
    if "table" in kw:
        tab = kw.pop("table")
    args = dict(sample_rate=44100.0, control_rate=441.0, noise_seed=0, mix_mode=0)
    args.update(kw)
    return _native.make_config(tab, **args)


def test_render_argument_checks_before_launch():
    cfg, keep = cfg_with()
    assert _render(None) == EINVAL
    assert _render(cfg, B=-1) == EINVAL
    assert _render(cfg, B=0) == 0                      # empty batch: no-op, no launch
    assert _render(cfg, params=None) == EINVAL
    assert _render(cfg, audio=None) == EINVAL
    assert _render(cfg, n=0) == EINVAL
    assert _render(cfg, rps=3) == EINVAL
    assert _render(cfg, slices=0) == EINVAL
    assert _render(cfg, n=100, slices=5) == EUNSUP     # more slices than chunks
    c2, k2 = cfg_with(mix_mode=2)
    assert _render(c2) == EINVAL
    c3, k3 = cfg_with(sample_rate=44100.0, control_rate=440.0)   # not an integer ratio
    assert _render(c3) == EUNSUP
    c4, k4 = cfg_with(sample_rate=4410.0, control_rate=441.0)    # q = 10, not a multiple of 4
    assert _render(c4) == EUNSUP
    bad = W.default_nebula().table()
    bad[5, 2] = 0.0                                     # curve must be > 0
    c5, k5 = cfg_with(table=bad)
    assert _render(c5) == EINVAL
    bad = W.default_nebula().table()
    bad[3, 3] = 0.5                                     # symmetric flag must be 0 or 1
    c6, k6 = cfg_with(table=bad)
    assert _render(c6) == EINVAL
    bad = W.default_nebula().table()
    bad[0, 0], bad[0, 1] = 90.0, 10.0                   # min > max
    c7, k7 = cfg_with(table=bad)
    assert _render(c7) == EINVAL
    cfg.reserved = 1
    assert _render(cfg) == EINVAL


def test_sample_params_argument_checks():
    L = _native.lib()
    assert L.synth_sample_params(0, 0, -1, None, 1, None) == EINVAL
    assert L.synth_sample_params(0, 0, 0, None, None, None) == 0
    assert L.synth_sample_params(0, 0, 5, None, None, None) == EINVAL


def test_mrstft_argument_checks_before_launch():
    """Rejected before any device work: bad sizes, missing buffers, a
    workspace that is not 16-byte aligned, more voices than the grid holds."""
    L = _native.lib()
    fake = ctypes.c_void_p(0x10000)            # never dereferenced on these paths
    odd = ctypes.c_void_p(0x10004)

    def call(B=2, n=4096, x=fake, t=fake, loss=fake, ws=fake, nbytes=1 << 40):
        return L.synth_mrstft_loss(x, t, B, n, loss, None, ws, nbytes, None)
    assert call(B=-1) == EINVAL
    assert call(n=0) == EINVAL
    assert call(x=None) == EINVAL
    assert call(ws=None) == EINVAL
    assert call(ws=odd) == EINVAL
    assert call(B=65536) == EUNSUP
    assert call(B=0) == 0
    assert call(nbytes=16) == -2                   # SYNTH_ENOMEM

    def cached(B=2, n=4096, x=fake, t=fake, tbytes=1 << 40, loss=fake, ws=fake, nbytes=1 << 40):
        return L.synth_mrstft_loss_cached(x, t, tbytes, B, n, loss, None, ws, nbytes, None)
    assert cached(B=-1) == EINVAL
    assert cached(t=None) == EINVAL
    assert cached(ws=odd) == EINVAL
    assert cached(B=65536) == EUNSUP
    assert cached(nbytes=16) == -2
    need = L.synth_mrstft_target_bytes(2, 4096)
    assert cached(tbytes=need - 1) == -2                  # target spectra of another size
    assert need > 0 and L.synth_mrstft_target_bytes(2, 300) == 0   # no frame fits
    assert L.synth_mrstft_target(fake, 2, 4096, fake, need - 1, None) == -2
    assert L.synth_mrstft_target(None, 2, 4096, fake, need, None) == EINVAL
    assert L.synth_mrstft_target(fake, 65536, 4096, fake, 1 << 40, None) == EUNSUP
    assert L.synth_mrstft_target(fake, 2, 300, None, 0, None) == 0


def test_binding_fails_loudly_without_library(tmp_path, monkeypatch):
    monkeypatch.setattr(_native, "LIB_PATH", str(tmp_path / "missing.so"))
    monkeypatch.setattr(_native, "_lib", None)
    with pytest.raises(ImportError):
        _native.lib()


def header_arities():
    """{name: number of parameters} of every function the headers declare."""
    out = {}
    for h in sorted(os.listdir(os.path.join(ROOT, "include"))):
        if not h.endswith(".h"):
            continue
        txt = open(os.path.join(ROOT, "include", h)).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        txt = re.sub(r"//[^\n]*", "", txt)
        for name, params in re.findall(r"\b(synth_[a-z0-9_]+)\s*\(([^()]*)\)\s*;", txt):
            params = params.strip()
            out[name] = 0 if params in ("", "void") else params.count(",") + 1
    return out


def test_ctypes_signatures_match_header_arity():
    """Every binding declares exactly the header's parameters: an argument past
    the declared list would be passed as a C int (a truncated stream pointer)."""
    from paper_2104_12922_amd import fm, learned, nebula, vcf
    L = learned.lib()
    for m in (fm, nebula, vcf):           # each module declares its entry points on first use
        assert m.lib() is L
    ar = header_arities()
    assert len(ar) == len(header_functions())
    for name, n in ar.items():
        at = getattr(L, name).argtypes
        assert at is not None, f"{name} has no argtypes"
        assert len(at) == n, f"{name}: header has {n} parameters, binding {len(at)}"
