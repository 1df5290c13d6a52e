"""sphx: SPH neighbour-loop hot path (density, ghost, force) for AMD MI355X.

The compute path is a C-ABI shared library of hand-written HIP kernels
(``libsphx.so``); ``paper_2305_13380_amd.sphx`` is its thin ctypes binding.
Importing this package loads nothing; importing ``.sphx`` loads the library
and fails loudly if it has not been built.
"""
__all__ = ["inputs"]
