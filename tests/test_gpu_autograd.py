"""Differentiation through the solver: the backward pass is the adjoint
multisplitting solve (A is symmetric).  Checked against the gradient of a
dense solve and against central finite differences.

L(f, g) = ||u - u_t||^2 with A u = h^2 f + lift(g) is quadratic in (f, g), so
central differences carry no truncation error; what is left is solver and
rounding noise, kept small by solving to tol 1e-13."""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs
from gpu_util import dev, host, say, torch_cuda
from oracle_pins import dense_laplacian

pytestmark = pytest.mark.gpu


def _problem(n, seed):
    rng = np.random.default_rng(seed)
    f = rng.standard_normal((n, n, n))
    g = inputs.random_faces(n, n, n, seed=seed + 1)
    ut = inputs.smooth_field((n, n, n), seed + 2)
    return f, g, ut


def _loss_and_grads(solver, f, g, ut):
    torch = torch_cuda()
    ft = dev(f).requires_grad_(True)
    gt = [dev(a).requires_grad_(True) for a in g]
    u = solver(ft, gt)
    L = ((u - dev(ut)) ** 2).sum()
    L.backward()
    return L.item(), host(ft.grad), [host(a.grad) for a in gt], host(u)


def test_adjoint_gradient_matches_dense_solve():
    from paper_2009_12638_amd.autograd import PoissonSolver
    n = 12
    f, g, ut = _problem(n, 50)
    solver = PoissonSolver((n, n, n), cuts=[[0, 6, 12]] * 3, tol=1e-13, inner_iters=10)
    say("autograd dense 12^3")
    L, gf, gg, u = _loss_and_grads(solver, f, g, ut)
    # dense reference
    A = dense_laplacian(n, n, n)
    h2 = (1.0 / (n + 1)) ** 2
    beff = h2 * f.copy()
    beff[0] += g[0]; beff[-1] += g[1]; beff[:, 0] += g[2]; beff[:, -1] += g[3]
    beff[:, :, 0] += g[4]; beff[:, :, -1] += g[5]
    uref = np.linalg.solve(A, beff.ravel()).reshape(n, n, n)
    lam = np.linalg.solve(A, 2 * (uref - ut).ravel()).reshape(n, n, n)
    assert np.linalg.norm(u - uref) <= 1e-10 * np.linalg.norm(uref)
    assert np.linalg.norm(gf - h2 * lam) <= 1e-9 * np.linalg.norm(h2 * lam)
    want_g = [lam[0], lam[-1], lam[:, 0], lam[:, -1], lam[:, :, 0], lam[:, :, -1]]
    for a, b in zip(gg, want_g):
        assert np.linalg.norm(a - b) <= 1e-9 * np.linalg.norm(b)


def test_adjoint_gradient_matches_finite_differences():
    torch = torch_cuda()
    from paper_2009_12638_amd.autograd import PoissonSolver
    n = 24
    f, g, ut = _problem(n, 60)
    solver = PoissonSolver((n, n, n), cuts=[[0, 12, 24]] * 3, tol=1e-13, inner_iters=10)
    say("autograd fd 24^3")
    L, gf, gg, _ = _loss_and_grads(solver, f, g, ut)
    uT = dev(ut)

    def loss(fv, gv):
        with torch.no_grad():
            u = solver(dev(fv), [dev(a) for a in gv])
            return float(((u - uT) ** 2).sum())

    hstep = 1e-6
    for j in range(8):
        rng = np.random.default_rng(53 + j)
        df = rng.standard_normal(f.shape)
        dg = [rng.standard_normal(a.shape) for a in g]
        lp = loss(f + hstep * df, [a + hstep * b for a, b in zip(g, dg)])
        lm = loss(f - hstep * df, [a - hstep * b for a, b in zip(g, dg)])
        fd = (lp - lm) / (2 * hstep)
        ad = float((gf * df).sum() + sum((a * b).sum() for a, b in zip(gg, dg)))
        assert abs(fd - ad) <= 1e-5 * max(abs(ad), 1e-3 * L), (j, fd, ad)
