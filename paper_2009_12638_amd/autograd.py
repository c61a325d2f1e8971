"""Differentiable Poisson solve through the multisplitting solver.

``PoissonSolve.apply(f, g0, ..., g5)`` returns u with ``A u = h^2 f + lift(g)``
(the 7-point operator of Section 2.1 of Brown, Bull and Bethune, solved by the
two-stage multisplitting of Section 3).  The backward pass is the adjoint
solve: A is symmetric, so the same solver applied to the incoming gradient
gives lambda = A^{-1} dL/du, and

* dL/df = h^2 * lambda;
* dL/dg (each boundary face) = lambda at the interior cells next to that
  face, because every face value enters b_eff exactly once, at its
  neighbouring cell (the 7-point stencil never touches edge or corner nodes).

All arithmetic runs on the GPU through the C ABI (the solves, the source
scaling h^2 f through ms_lift on the handle with zero boundary data, and the
parameter gradients through ms_lift_adjoint); this module only allocates and
moves tensors.
"""
from __future__ import annotations

import torch

from . import ms


class PoissonSolver:
    """Owns a handle for the forward solve (boundary data set per call) and one
    with zero boundary data for the adjoint solve.  adjoint_tol (default tol)
    is the relative residual the adjoint solve stops at: its solution can be
    far larger than its right-hand side (up to 1/lambda_min times), which
    raises the FP64 residual floor of that solve above the forward one's.
    overlap > 0 solves both on overlapping blocks of that depth.  stats holds
    the ms.Stats of the last forward and adjoint solves."""

    def __init__(self, shape, blocks=None, cuts=None, tol=1e-12, inner_iters=10,
                 precision="fp64", mode="sync", max_sweeps=200000, adjoint_tol=None,
                 overlap=0):
        self.shape = tuple(int(s) for s in shape)
        self.h_fwd = ms.ms_create(self.shape, blocks=blocks, cuts=cuts)
        self.h_adj = ms.ms_create(self.shape, blocks=blocks, cuts=cuts)
        if overlap:
            ms.ms_set_overlap(self.h_fwd, int(overlap))
            ms.ms_set_overlap(self.h_adj, int(overlap))
        self.tol = tol
        self.adjoint_tol = tol if adjoint_tol is None else adjoint_tol
        self.m = inner_iters
        self.precision = precision
        self.mode = mode
        self.max_sweeps = max_sweeps
        self.spacing = 1.0 / (self.shape[0] + 1)
        self.stats = {}

    def _solve(self, handle, rhs, tol, which):
        x = torch.zeros(self.shape, dtype=torch.float64, device=rhs.device)
        self.stats[which] = ms.ms_solve(handle, rhs.contiguous(), x, tol, self.m, self.mode,
                                        precision=self.precision, max_sweeps=self.max_sweeps)
        return x

    def __call__(self, f, faces):
        return PoissonSolve.apply(self, f, *faces)


class PoissonSolve(torch.autograd.Function):
    @staticmethod
    def forward(ctx, solver: PoissonSolver, f, *faces):
        h2 = solver.spacing ** 2
        face_list = [None if g is None else g.detach().contiguous() for g in faces]
        ms.ms_set_bc(solver.h_fwd, face_list)
        rhs = torch.empty(solver.shape, dtype=torch.float64, device=f.device)
        # h^2 f (the adjoint handle has zero boundary data, so nothing is lifted)
        ms.ms_lift(solver.h_adj, f.detach().contiguous(), h2, rhs)
        u = solver._solve(solver.h_fwd, rhs, solver.tol, "forward")
        ctx.solver = solver
        ctx.has_face = [g is not None for g in faces]
        return u

    @staticmethod
    def backward(ctx, grad_u):
        solver = ctx.solver
        lam = solver._solve(solver.h_adj, grad_u.detach().contiguous(), solver.adjoint_tol,
                            "adjoint")
        h2 = solver.spacing ** 2
        nx, ny, nz = solver.shape
        face_shapes = [(ny, nz), (ny, nz), (nx, nz), (nx, nz), (nx, ny), (nx, ny)]
        grad_f = torch.empty_like(lam)
        # dL/dg for the faces -x, +x, -y, +y, -z, +z (those that were given)
        grad_g = [torch.empty(fs, dtype=torch.float64, device=lam.device) if has else None
                  for fs, has in zip(face_shapes, ctx.has_face)]
        ms.ms_lift_adjoint(solver.h_adj, lam, h2, grad_f, grad_g)
        return (None, grad_f, *grad_g)
