"""MI355X-native APRIL intermediate filter (raster interval lists).

The compute lives in libapril.so (HIP kernels for gfx950 behind the C ABI in
include/april.h); `paper_2307_01716_amd.april` is its ctypes binding.
"""
