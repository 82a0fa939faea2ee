"""MI355X (gfx950) library for the data-parallel online phase of SPDZ.

The compute path is libspdz.so (HIP kernels behind the C ABI in
include/spdz.h); `spdz` is its ctypes binding.
"""
from . import spdz  # noqa: F401
