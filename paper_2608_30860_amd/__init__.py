"""lindx: steady states, low-lying spectra and steady-state gradients of Lindblad equations on
AMD Instinct MI355X (gfx950), built on the map Phi = -K S^{-1} of arXiv 2608.30860.

The compute path is the HIP library liblindx.so (C ABI in include/lind.h); this package holds
its build script and a thin ctypes binding on torch tensors.  Importing the package does not
load the library; constructing a ``Lindblad`` does, and fails loudly if it is not built or no
gfx950 device is present.
"""
from .lindx import (Lindblad, LindError, SteadyExpect, load_library, steady_expectation,  # noqa: F401
                    LIB_PATH, SYMBOLS, PREC, ROUTE)
