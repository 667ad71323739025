"""MI355X-native ADMM distributed bundle adjustment (gfx950 HIP kernels
behind a C ABI, include/dba.h).  ``binding`` is the ctypes layer."""
from . import binding  # noqa: F401
from .binding import Solver, DbaError  # noqa: F401
