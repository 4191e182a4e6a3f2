"""Plain FP64 CPU oracle for nodal DG Maxwell on tetrahedra.

TEST INFRASTRUCTURE ONLY. Nothing in the product path imports, calls or executes this package;
only the tests, `__graft_entry__.smoke()` and the CPU-baseline leg of `bench.py` do.

The oracle is the plain definition of the semi-discrete operator of Sec. 2 (eqs. strong-dg and
semidiscrete-dg, the reference matrices of eq. dg-reference-matrices) specialised to Maxwell's
equations with the upwind flux of Sec. 6, plus the five-stage low-storage RK4 time stepper
named in Sec. 6. It is written with NumPy (library matmuls, solves and eigenvalue routines as
steps) and shares no code with the HIP path or its C++ host builder.

Modules:
  refelem  reference tetrahedron: warp-and-blend nodes, orthonormal basis, D, LIFT
  mesh     orientation, face connectivity, geometric factors, normals, coordinate face maps
  maxwell  right-hand side, LSRK4, energy, time step
"""
from . import refelem, mesh, maxwell  # noqa: F401
