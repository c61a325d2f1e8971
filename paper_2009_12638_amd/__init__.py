"""Two-stage multisplitting (block Jacobi outer sweep, CG inner solves) for
the 3D 7-point Laplace/Poisson system on AMD Instinct MI355X (gfx950).

The solver is the HIP library ``libms.so`` built from ``csrc/``; ``ms`` is
its thin ctypes binding (same entry-point names as ``include/ms.h``) and
``inputs`` holds the seeded workload generators.  Importing the package loads
nothing; the library is opened on first use and its absence is an error.
"""
__all__ = ["ms", "inputs"]
__version__ = "0.1.0"
