"""MI355X-native short-range pair-force engine (vertex and edge decompositions).

The compute path lives in ``libmd.so`` (hand-written HIP for gfx950 behind a
C ABI, declared in ``include/md.h``).  ``paper_1401_4350_amd.md`` is the thin
ctypes binding; importing it loads the library and raises if it is missing.
"""
__all__ = ["inputs", "md"]
