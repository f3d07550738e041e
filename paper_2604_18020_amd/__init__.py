"""MI355X (gfx950) matrix-free 3D SIMP topology optimisation.

The compute path is the HIP library libtosimp.so (C ABI in include/tosimp.h); this
package is its thin binding.  Import it with the library built in-tree:

    python paper_2604_18020_amd/build.py
"""
from .binding import (F32, F64, PREC, Tosimp, TosimpError, tridiag_extremes,  # noqa: F401
                      version, LIB_PATH, OK, NOT_CONVERGED, FALLBACK_USED)
