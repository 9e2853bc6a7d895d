"""MI355X-native ROI reduction of X-CT volumes (ROIX-Comp, arXiv 2602.15917).

Error-bounded quantisation, Otsu threshold + 3-D connected components, and
compaction of the retained rows into a packed code stream, as hand-written
HIP kernels for gfx950 behind the C ABI in include/roix.h.  ``roix`` is the
ctypes binding; ``build`` compiles the library.
"""
from . import roix  # noqa: F401

__all__ = ["roix"]
