"""MI355X-native D2V16 MRT finite-difference lattice Boltzmann solver.

The hot path (moments, equilibrium moments, M / relax / Minv collision,
Lax-Wendroff convection and forward-Euler advance, boundary ghosts) runs in
hand-written HIP kernels for gfx950 behind the C ABI declared in
``include/mrtlb.h``; this package is its thin Python binding.  Submodules are
imported lazily so that ``workloads`` (seeded inputs, no scheme arithmetic)
can be used without the compiled library.
"""
__all__ = ["lib", "solver", "batch", "adjoint", "workloads"]
