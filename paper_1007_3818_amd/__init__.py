"""MI355X (gfx950) MUSCL-Hancock + Roe hydro solver for batches of ghost-padded
16^3 patch groups, behind the C ABI of include/gamer_hydro.h.

Modules:
  hydro      torch-tensor front end of the C ABI (device memory and streams only)
  stepper    multi-step drivers (periodic uniform grid, batched AMR-like levels,
             HIP-graph captured steps)
  workloads  seeded synthetic initial conditions
  build      in-tree build of libgamer_hydro.so
Importing the package does not load the native library; the first call does,
and fails loudly if it has not been built.
"""
__all__ = ["hydro", "workloads", "build", "stepper"]
