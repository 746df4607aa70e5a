"""Constant-memory differentiable light tracing on MI355X (gfx950).

Submodules:
  scenes  seeded synthetic scene generators (inputs only)
  lt      ctypes binding of the HIP C-ABI library (liblt.so) and the
          torch.autograd.Function wrappers
"""
