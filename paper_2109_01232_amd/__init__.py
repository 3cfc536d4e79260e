"""MI355X-native GMRES-IR: mixed-precision restarted GMRES with iterative refinement.

The solver (CSR SpMV, two-pass classical Gram-Schmidt, Givens least squares,
fp64 residual and correction, polynomial preconditioner, chooser network) is
hand-written HIP for gfx950 in ``csrc/`` behind the C ABI of
``include/gmresir.h``; ``binding`` is its ctypes binding.  ``problems``
builds the seeded synthetic test systems.  Nothing here imports the library
at package import time; ``binding.lib()`` loads it on first use.
"""

__all__ = ["binding", "problems", "build"]
