"""MI355X-native decoupled correlative pose search (Fast-MbyM).

The search runs in hand-written HIP kernels behind the C ABI of ``libfmbym.so``
(declared in ``include/fmbym.h``).  ``fmbym`` is the thin ctypes binding; it is
imported lazily so that the input generator in ``synth`` can be used without
loading the library.
"""
__all__ = ["synth", "fmbym"]


def __getattr__(name):
    if name == "fmbym":
        from . import fmbym as _f
        return _f
    if name == "synth":
        from . import synth as _s
        return _s
    raise AttributeError(name)
