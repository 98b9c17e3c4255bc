"""MI355X-native primal-dual domain decomposition for dual total-variation problems.

The solver (Lee & Park, arXiv 1901.00682, Algorithm 1) runs in hand-written
HIP kernels for gfx950 behind the C-ABI library ``libdtvdd.so``; this package
is the thin Python binding over it.  Submodules are imported lazily so that
``synth`` (input generation) works without the native library.
"""
__all__ = ["dtvdd", "synth"]
