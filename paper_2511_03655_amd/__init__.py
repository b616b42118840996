"""MI355X-native fixed-step IRKGL16 (8-stage Gauss-Legendre collocation, order
16) for separable second-order Hamiltonian systems q'' = g(q), in FP64, in the
floating-point-symplectic second-order formulation with compensated
summation of the state.

The integrator runs entirely in hand-written HIP kernels for gfx950 behind the
C-ABI library ``libirkgl16.so`` (see ``include/irkgl16.h``); this package is a
thin ctypes binding plus seeded workload generators.
"""
