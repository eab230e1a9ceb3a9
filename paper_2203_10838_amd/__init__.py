"""gfx950 implementation of the averaged randomized sparse Kaczmarz method (RSKA).

Submodules:
  rsk     -- Python binding of librsk (HIP kernels behind the C ABI in include/rsk.h)
  inputs  -- seeded synthetic inputs (no arithmetic of the method)
  params  -- parameter formulas of the paper (optimal relaxation)
  build   -- in-tree hipcc build of librsk.so
"""
__all__ = ["rsk", "inputs", "params", "build"]
