"""MI355X-native lattice Dirac-operator solvers (liblq) and their Python binding.

The product is the HIP library liblq.so (include/lq.h); `lq` is its ctypes
binding.  Build it with `python -m paper_2201_09004_amd.build`.
"""
from . import lq  # noqa: F401

__all__ = ["lq"]
