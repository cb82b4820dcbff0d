"""MI355X (gfx950) PSATD Maxwell step with guard cells: HIP kernels behind a C ABI.

The compute path lives in libpsatd.so (paper_1812_07357_amd/csrc, declared in
include/psatd.h); ``psatd`` is its ctypes binding.  Importing ``psatd`` fails
loudly if the library has not been built.
"""

__all__ = ["psatd"]
