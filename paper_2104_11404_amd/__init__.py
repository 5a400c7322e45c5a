"""MI355X-native hyper-reduced Lagrangian-hydrodynamics ROM (arXiv 2104.11404).

The computation lives in ``liblagrom.so`` (hand-written HIP for gfx950 behind
the C ABI declared in ``include/lagrom.h``).  ``lib`` is a thin ctypes
binding with the same names; ``build`` compiles the library in-tree.
"""
