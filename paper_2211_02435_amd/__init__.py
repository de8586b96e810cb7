"""MI355X (gfx950) zero-centred MRT lattice Boltzmann library.

The computation lives in libpaper_lbm.so (HIP kernels behind the C ABI of include/lbm.h);
`lbm` is its ctypes binding.  Importing the package does not touch the GPU.
"""
from . import lbm  # noqa: F401

__all__ = ["lbm"]
