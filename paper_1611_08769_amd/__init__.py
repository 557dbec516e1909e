"""Encrypted fixed-point FFT over GSW13 on MI355X (gfx950).

Submodules:
  sfft       -- ctypes binding of libsfft (include/sfft.h)
  api        -- keys / encryption / plans / decryption with torch device memory
  workloads  -- seeded synthetic signals and images
  build      -- in-tree build of libsfft.so
"""
