"""MI355X-native sparse spectral Galerkin solver for -div(a grad u) = f on the d-torus.

* ``sparsespec`` -- ctypes binding of the HIP library ``libsparsespec.so``
  (stamp sets, neighbour map, SELL-64 matvec, batched PCG, FP32+FP64
  refinement).  Importing it requires the built library.
* ``serving``    -- continuous-batching request loop over the library.
* ``workloads``  -- seeded synthetic PDE data.
* ``build``      -- compiles the HIP sources for gfx950.
"""
__all__ = ["sparsespec", "workloads", "build", "serving"]
