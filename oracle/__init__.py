"""CPU oracle of the modular-synth voice render (arXiv 2104.12922).

TEST INFRASTRUCTURE ONLY.  Only ``tests/``, ``__graft_entry__.smoke()`` and the
CPU-baseline leg of ``bench.py`` may import anything from this package.  The
product path (``paper_2104_12922_amd``) never imports it and shares no code
with it; both sides read only the seeded inputs defined in ``workloads``.

The oracle is plain, slow and written for a reader to check against the paper:
float64 throughout (torch CPU tensors, so that autograd also yields the
oracle's exact gradient), one function per module of the Voice (Section 3.2),
each module in signal order.

Modules
-------
philox   Philox4x32-10 counter-based generator (Salmon et al., SC 2011), used
         for the deterministic parameter draw and the noise oscillator
         (Section 2.1: deterministic RNG "even of noise oscillators").
voice    vectorised float64 Voice render (Sections 3.1-3.3).
brute    scalar pure-Python Voice render for tiny inputs (pins ``voice``).
spectral STFT, multi-resolution log-magnitude STFT L1 and log-mel features.
mlp      the learned proposal's MLP forward/backward and Adam.
mmd      maximum mean discrepancy between sets of sounds (Section 5) with the
         L1 distance between log-mel embeddings.

Parity status
-------------
Every definition the paper leaves to torchsynth's code and documentation (the
exact ADSR, LFO, square-saw and mixer formulas, the RNG streams) is a reading
of the paper's prose; sample parity with the published synth1B1 corpus is therefore
"parity unpinned" and not claimed.  Each stage is pinned by closed forms and
invariants in ``tests/test_oracle_*.py``.
"""
