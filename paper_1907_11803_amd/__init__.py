"""MI355X-native engine for p-stable LSH similarity-search query workloads.

Submodules:
  lib    -- ctypes binding of libqwlsh.so (the C ABI declared in include/qwlsh.h)
  synth  -- seeded synthetic workloads (input recipes only)
  build  -- compiles the HIP sources for gfx950 into libqwlsh.so

Importing the package loads nothing; `lib.load()` (called by every binding
function) raises if the library has not been built.
"""

__all__ = ["lib", "synth", "build"]
