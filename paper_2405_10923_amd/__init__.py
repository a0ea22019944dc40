"""MI355X (gfx950) randomized Householder QR: HIP kernels behind a C ABI
(include/rhqr.h, librhqr.so) with a thin ctypes binding (``rhqr``)."""
from . import rhqr  # noqa: F401
