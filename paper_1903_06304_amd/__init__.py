"""MI355X-native implicit Weiss-Smith-preconditioned FR/CPR hot path (HIP, gfx950).

Submodules:
  inputs  -- seeded synthetic meshes and initial fields (no method arithmetic)
  lmfr    -- ctypes binding of the C ABI in include/lmfr.h (loads liblmfr.so)
  build   -- hipcc build of liblmfr.so
The binding is imported on demand so that importing the package never needs a GPU.
"""
__all__ = ["inputs", "lmfr", "build"]
