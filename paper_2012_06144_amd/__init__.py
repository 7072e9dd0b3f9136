"""MI355X-native coupled conservative Allen-Cahn phase-field (D3Q15) and
velocity-based hydrodynamic (D3Q27) lattice Boltzmann step (Holzer et al.,
IJHPCA 2020), as hand-written HIP sweeps behind a C ABI.

Submodules:
  lbm     -- ctypes binding of liblbm.so (the GPU solver)
  inputs  -- seeded synthetic initial conditions
  build   -- compiles the HIP library for gfx950
The binding is imported lazily so ``inputs`` works without a GPU build.
"""
__all__ = ["lbm", "inputs", "build"]
