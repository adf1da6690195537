"""MI355X-native domain-decomposed Wilson-clover propagators (libddml).

The compute path is the HIP library libddml.so (csrc/, C ABI in
include/ddml.h); this package holds its build script and the thin ctypes
binding ``ddml``.
"""
from . import ddml  # noqa: F401
