"""MI355X-native hot path of CUBE's information-optimised particle-mesh step (arXiv:1712.06121).

The product is libcube.so (HIP kernels for gfx950 behind the C ABI in include/cube.h); this
package holds its sources (csrc/), the in-tree build (build.py) and the ctypes binding
(binding.py). Importing the package does not load the library; ``Sim`` does, and fails loudly
when the library has not been built.
"""
from .binding import (CUBE_DONE, CUBE_OK, EXPORTED, LIB_PATH, SIGMA_GLOBAL, SIGMA_PER_CELL, Batch, CubeError, Server,
                      Sim, counts_from_u8, footprint, load_library, make_params)

__all__ = ["Sim", "Batch", "Server", "CubeError", "counts_from_u8", "footprint", "load_library", "make_params", "LIB_PATH", "EXPORTED",
           "SIGMA_GLOBAL", "SIGMA_PER_CELL", "CUBE_OK", "CUBE_DONE"]
