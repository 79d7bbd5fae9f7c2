"""MI355X solver for repeated 2D FDFD solves with cached factorisations.

Submodules:
  problems  seeded synthetic workloads (inputs only)
  build     compiles libfdfd.so (hipcc, gfx950)
  fdfd      ctypes binding of the C ABI (Plan)
  autograd  torch.autograd.Function over the solver
"""
__all__ = ["problems", "build", "fdfd", "autograd"]
