"""Oracle of the D2V16 MRT finite-difference lattice Boltzmann scheme (plain FP64, CPU).

TEST INFRASTRUCTURE ONLY.  This package is the independent reference that the
HIP path is checked against.  Only the test suite, the smoke check of
``__graft_entry__`` and the CPU-baseline leg of ``bench.py`` may import it; the
product package never does, and it imports nothing from the product package.

Modules
-------
mrt        the scheme itself: velocity set, transformation matrix, equilibrium
           moments, collision, Lax-Wendroff convection, ghost layers, time step
adjoint    discrete adjoint of one time step and of the initialisation, by
           complex-step differentiation of the functions in ``mrt``
riemann    exact solution of the 1D Riemann problem of the Euler equations
stability  linear (von Neumann) amplification spectrum of the scheme
"""
