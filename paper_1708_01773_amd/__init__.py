"""MI355X-native finite element hot path: Q_k integration, deterministic CSR
scatter and Jacobi-PCG, as HIP kernels behind the C ABI of include/fe.h.

Importing the package loads the built library (libfe.so) and fails loudly if
it is missing; build it with ``__graft_entry__.build()``.
"""
from . import fe  # noqa: F401
from .fe import (Assembly, FeError, Mesh, assemble, assemble_query, create_mesh, make_coeff,  # noqa: F401
                 pcg_query, pcg_solve, spmv)

fe.lib()
