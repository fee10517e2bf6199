"""Gradient-type subspace iteration (Riemannian steepest descent and nonlinear CG with an
exact line search) for the dominant invariant subspace of a sparse symmetric matrix, as
hand-written HIP kernels for MI355X (gfx950) behind a C ABI.

Submodules:
  inputs -- seeded synthetic problems and starting blocks (no solver arithmetic)
  gsi    -- ctypes binding of the C ABI (loads libgsi.so; raises if it is missing)
"""
