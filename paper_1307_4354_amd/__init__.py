"""MI355X (gfx950) Closest Point Method multigrid solver for elliptic equations on
surfaces (Chen & Macdonald): hand-written HIP kernels behind the C ABI of libcpm.so,
with a thin ctypes binding that keeps the C names.  The package refuses to import when
the native library is missing."""
from .binding import *  # noqa: F401,F403
from .binding import Band, CpmError, LIB_PATH, make_params, make_surface  # noqa: F401
