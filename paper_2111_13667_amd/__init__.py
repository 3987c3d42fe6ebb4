"""MI355X-native batched transfer-matrix evaluation (R, T, r, t for s and p).

The compute path is ``libtmm_rt.so`` (hand-written HIP for gfx950 behind a C
ABI, declared in ``include/tmm_rt.h``); ``tmm`` is the thin ctypes binding.
Importing this package loads nothing: the library is opened on first use and a
missing library is an error, never a fallback.
"""
__all__ = ["workloads", "tmm"]
