"""Two-stage multisplitting (block Jacobi outer sweeps, synchronous or
asynchronous, with CG or GMRES inner solves on plain or overlapping blocks)
for the 3D 7-point Laplace/Poisson system on AMD Instinct MI355X (gfx950).

The solver is the HIP library ``libms.so`` built from ``csrc/``.  Modules:

* ``ms``: thin ctypes binding, same entry-point names as ``include/ms.h``;
* ``autograd``: a differentiable solve whose backward pass is the adjoint
  solve;
* ``tune``: tile/grouping, inner-iteration and overlap tuning, and
  inner-iteration schedules;
* ``inputs``: the seeded workload generators.

Importing the package loads nothing; the library is opened on first use and
its absence is an error.
"""
__all__ = ["ms", "inputs", "autograd", "tune"]
__version__ = "0.1.0"
