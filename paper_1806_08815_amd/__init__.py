"""dapt: the Digital Annealer's parallel-trial Monte Carlo step, native to MI355X.

The compute path is a C-ABI shared library of hand-written HIP kernels for
gfx950 (``csrc/``, declared in ``include/da.h``); ``api`` is a thin ctypes
binding with the same names.  ``instances`` and ``workloads`` build seeded
synthetic inputs; ``tts`` is the time-to-solution analysis.
"""
__all__ = ["api", "instances", "workloads", "tts"]
