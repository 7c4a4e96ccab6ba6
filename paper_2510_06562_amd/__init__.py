"""MI355X-native hot path of distilled multi-time-step (DMTS) molecular dynamics.

The compute path is a C-ABI shared library of hand-written HIP kernels for gfx950
(``csrc/``); ``api`` binds it with ctypes.  ``synth`` holds the seeded input generators.
Importing the package loads nothing; the library is loaded on first use of ``api``.
"""

__all__ = ["api", "synth"]
