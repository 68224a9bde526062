"""MI355X-native decoupled correlative pose search (Fast-MbyM).

The search runs in hand-written HIP kernels behind the C ABI of ``libfmbym.so``
(declared in ``include/fmbym.h``).  Submodules: ``fmbym`` (the thin ctypes
binding, which loads the library), ``synth`` (seeded input generator) and
``workloads`` (parameter sets).  Importing the package loads nothing.
"""
