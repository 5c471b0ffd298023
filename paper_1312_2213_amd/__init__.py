"""MI355X-native parallel multicanonical (MUCA/MUMA) simulations.

The hot path lives in libmuca.so (HIP kernels for gfx950 plus the C ABI of
include/muca.h); ``paper_1312_2213_amd.muca`` is its ctypes binding.
"""
