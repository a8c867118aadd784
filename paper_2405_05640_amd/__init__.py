"""MI355X-native spectral-element pressure-solve hot path.

``sem``        -- ctypes binding of the HIP library libsem.so (C ABI in include/sem.h)
``workloads``  -- seeded synthetic meshes and right-hand sides
``build``      -- in-tree hipcc build of libsem.so for gfx950
"""
