"""MI355X-native engine for the vectorial lattice Boltzmann scheme.

The compute path is the HIP library liblbm.so (csrc/, C ABI in include/lbm.h);
`lbm` is its ctypes binding.  torch supplies device memory and streams only.
"""

from . import batch, closure, cnn, lbm  # noqa: F401

__all__ = ["lbm", "batch", "cnn", "closure"]
