"""MI355X (gfx950) FFT spectral-block library.

Submodules:
  fb      -- ctypes binding of libfb.so (the C ABI in include/fb.h)
  inputs  -- seeded synthetic inputs (SplitMix64 uniform / Box-Muller)
  build   -- in-tree build of libfb.so with hipcc
"""
__all__ = ["fb", "inputs", "build"]
