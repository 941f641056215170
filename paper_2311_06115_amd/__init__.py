"""MI355X-native hierarchical diffusion maps (the GOFMM-style H-matrix eigensolve of arXiv 2311.06115).

The computation lives in libhdm.so (HIP, gfx950) behind the C ABI of
include/hdm.h; ``hdm`` is its ctypes binding.
"""
