"""MI355X (gfx950) Monte Carlo solver for the gravity forward problem by the
Feynman-Kac formula (arXiv:1709.07469), behind the C interface of
include/fkgrav.h.

Modules:
  fkgrav     ctypes binding of libfkgrav.so (the HIP library)
  build      hipcc build of libfkgrav.so
  workloads  seeded synthetic problems (inputs only)
"""
__all__ = ["fkgrav", "build", "workloads"]
