"""MI355X-native Multipole-Accelerated Hamiltonian Interpolation (MAHI).

The compute path is libmahi.so (HIP kernels for gfx950, C ABI in
include/mahi.h); this package is its Python binding.
"""
from .mahi import (Batch, Mahi, MahiError, autotune, device_selftest, dlambda, from_system, host_selftest,  # noqa: F401
                   site_extent,
                   lambda_tilde, lib)
