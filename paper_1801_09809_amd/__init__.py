"""MI355X-native heavy-weight perfect matching (HWPM).

The hot path -- the bulk-synchronous weight-increasing 4-cycle rounds of
Azad et al. (arXiv 1801.09809, Section 5.3) -- runs as hand-written HIP
kernels in libhwpm.so behind the C ABI of include/hwpm.h; `hwpm` is its thin
ctypes binding.
"""
from .build import LIB, build_library  # noqa: F401
