"""MI355X (gfx950) implementation of the PCEXP exponential-integrator hot path
for DG-discretised Euler equations (arXiv 1801.06300).

The compute path is libpcexp.so (HIP kernels behind the C ABI of
include/pcexp.h); :mod:`paper_1801_06300_amd.binding` is a thin ctypes
binding over it.  Nothing here falls back to CPU code.
"""

from .binding import PCEXP, PcexpError, load_library, LIB_PATH  # noqa: F401
