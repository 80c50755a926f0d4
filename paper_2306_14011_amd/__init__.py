"""MI355X-native explicit finite-volume Euler step with ML launch autotuning.

The compute path is the HIP library ``libfv.so`` (hand-written gfx950 kernels
behind the C ABI declared in ``include/fv.h``); ``fv`` is its thin ctypes
binding. Importing this package loads nothing: the library is opened on first
use of ``paper_2306_14011_amd.fv`` and raises if it has not been built.
"""

__all__ = ["inputs", "fv"]
