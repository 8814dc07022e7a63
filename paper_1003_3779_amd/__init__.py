"""MI355X-native coined quantum-walk engine (arXiv:1003.3779).

The compute path lives in ``libqwalk.so`` (HIP kernels for gfx950 behind a
C ABI, declared in ``include/qwalk.h``); ``paper_1003_3779_amd.qwalk`` is the
thin ctypes binding.  Importing this package loads nothing: the library is
opened on first use of the binding.
"""
__all__ = ["qwalk", "inputs"]
