"""MI355X (gfx950) implementation of the upscaled Brinkman lattice Boltzmann
method of Li and Brown (arXiv:1312.0195).

Modules:
  lbm     -- ctypes binding of liblbm.so (the HIP kernels behind a C ABI)
  inputs  -- seeded synthetic permeability fields and patch lists
  build   -- compiles liblbm.so with hipcc for gfx950

Importing the package loads nothing; lbm.lib() loads the library and fails
loudly when it has not been built.
"""
__all__ = ["lbm", "inputs", "build"]
