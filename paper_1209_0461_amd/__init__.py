"""MI355X (gfx950) particle-mesh gravity step with linear-response massive neutrinos.

The step (CIC deposit, FFT, FP64 k-binning, the neutrino history integral, rescale,
Green's function, gradient, inverse FFT, CIC interpolation) runs in the hand-written HIP
kernels of libpmnu.so behind the C ABI of include/pm_nu.h; this package is its ctypes
binding. Build the library with ``python -m paper_1209_0461_amd.build``.
"""
from .binding import (PMNu, PMNuError, Config, load_library, LIB_PATH,  # noqa: F401
                      SIGNATURES)
from . import binding  # noqa: F401
