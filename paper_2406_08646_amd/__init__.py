"""MI355X-native COO assembly, CSR products and Jacobi-PCG (arXiv 2406.08646 hot path).

Submodules:
  spx        ctypes binding of the C ABI in include/spx.h (loads _lib/libspx.so)
  autograd   torch.autograd.Function for u = A(v)^-1 b with an adjoint backward
  autotune   launch-shape search for the batched solver
  workloads  seeded synthetic inputs (no method arithmetic)
  build      compiles the HIP sources into _lib/libspx.so

Importing the package loads nothing native; the binding loads the library on
first use and raises if it has not been built.
"""

__all__ = ["spx", "autograd", "autotune", "workloads", "build"]
