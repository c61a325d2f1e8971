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


@pytest.mark.parametrize("overlap,precision", [(0, "fp64"), (2, "fp64"), (2, "mixed")])
def test_adjoint_gradient_matches_dense_solve(overlap, precision):
    """Forward and adjoint solves (plain or overlapping blocks, FP64 or mixed
    refinement) against the dense solve's gradient; the solver reports both
    solves' stats."""
    from paper_2009_12638_amd.autograd import PoissonSolver
    n = 12
    f, g, ut = _problem(n, 50)
    solver = PoissonSolver((n, n, n), cuts=[[0, 6, 12]] * 3, tol=1e-13, inner_iters=10,
                           overlap=overlap, precision=precision)
    say("autograd dense 12^3", overlap, precision)
    L, gf, gg, u = _loss_and_grads(solver, f, g, ut)
    assert set(solver.stats) == {"forward", "adjoint"}
    assert all(st.status == 0 and st.rel_residual <= 1e-13 for st in solver.stats.values())
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


# --------------------------------------------------------------------------
# Full-size differentiation workload: 128^3, 4^3 blocks of 32^3, 64 seeded
# directions, central differences with step 1e-6 in FP64.
# --------------------------------------------------------------------------

DIFF_DIRECTIONS = 64
DIFF_CHUNKS = 4          # 16 directions = 32 right-hand sides per batched solve
DIFF_STEP = 1e-6
DIFF_TOL = 1e-14         # perturbed solves; the residual floor here is ~1e-16
_diff = {}


def _lambda_min(n):
    """Smallest eigenvalue of the 7-point operator on an n^3 grid."""
    return 3.0 * (2.0 - 2.0 * np.cos(np.pi / (n + 1)))


def _diff_point():
    """Forward solve and adjoint gradient at the workload's (f, g), once."""
    if not _diff:
        torch = torch_cuda()
        from paper_2009_12638_amd.autograd import PoissonSolver
        w = inputs.workload("diff128")
        cuts = [list(map(int, c)) for c in w["cuts"]]
        solver = PoissonSolver(w["shape"], cuts=cuts, tol=w["tol"], inner_iters=w["m"],
                               adjoint_tol=w["adjoint_tol"])
        say("autograd diff128 forward + adjoint")
        ft = dev(w["f"]).requires_grad_(True)
        gt = [dev(a).requires_grad_(True) for a in w["faces"]]
        u = solver(ft, gt)
        ut = dev(w["ut"])
        L = ((u - ut) ** 2).sum()
        L.backward()
        # achieved residuals of the two solves (forward with faces, adjoint)
        from paper_2009_12638_amd import ms
        h2 = solver.spacing ** 2
        _diff.update(w=w, cuts=cuts, u=u.detach(), ut=ut, L=L.item(), h2=h2,
                     gf=host(ft.grad), gg=[host(a.grad) for a in gt],
                     res_u=ms.ms_residual(solver.h_fwd, (h2 * ft.detach()).contiguous(),
                                          u.detach())[1],
                     res_lam=ms.ms_residual(solver.h_adj, (2 * (u - ut)).detach().contiguous(),
                                            dev(np.asarray(ft.grad.cpu()) / h2))[1])
    return _diff


@pytest.mark.parametrize("chunk", range(DIFF_CHUNKS))
def test_diff128_adjoint_matches_finite_differences(orc, chunk):
    """dL/df and dL/dg from the adjoint solve against central differences of
    L on seeded directions (both parts, source only, faces only).  Each
    perturbed loss comes from a batched FP64 solve of
    A x = lift(h^2 (f +- s df), g +- s dg) to tol 1e-14, warm-started from the
    forward solution.

    L is quadratic, so central differences have no truncation error; the
    bound below is what solver residuals can produce.  With A symmetric
    positive definite, a residual rho gives an error of at most
    rho / lambda_min, so for x with residual rho:
      |L(x) - L(u)| <= 2 ||u - u_t|| e + e^2,  e = rho / lambda_min,
    and the adjoint directional derivative b_v . lambda errs by at most
    ||b_v|| (rho_lambda + 2 rho_u) / lambda_min, b_v = lift(h^2 df, dg).
    A rounding allowance of 1e-14 L / s covers the FP64 sums of L."""
    torch = torch_cuda()
    from paper_2009_12638_amd import ms
    D = _diff_point()
    w = D["w"]
    shape, n, s, h2 = w["shape"], w["shape"][0], DIFF_STEP, D["h2"]
    lam_min = _lambda_min(n)
    per = DIFF_DIRECTIONS // DIFF_CHUNKS
    js = list(range(chunk * per, (chunk + 1) * per))
    B = torch.empty((2 * per,) + shape, dtype=torch.float64, device="cuda")
    bv_norm = []
    for k, j in enumerate(js):
        df, dg = inputs.diff_direction(shape, j)
        for sign, slot in ((1.0, 2 * k), (-1.0, 2 * k + 1)):
            fb = h2 * (w["f"] + sign * s * df)
            gb = [a + sign * s * b for a, b in zip(w["faces"], dg)]
            B[slot] = dev(orc.lift_bc(fb, gb))
        bv_norm.append(np.linalg.norm(orc.lift_bc(h2 * df, dg)))
    X = D["u"].unsqueeze(0).repeat(2 * per, 1, 1, 1).contiguous()
    hb = ms.ms_create(shape, cuts=D["cuts"])
    ms.ms_reserve(hb, 2 * per)
    say("autograd diff128 fd chunk", chunk, "directions", js[0], "to", js[-1])
    stats = ms.ms_solve_batch(hb, B, X, DIFF_TOL, w["m"], max_sweeps=20000, precision="fp64")
    ms.ms_destroy(hb)
    bnorm = torch.linalg.vector_norm(B.reshape(2 * per, -1), dim=1).cpu().numpy()
    losses = ((X - D["ut"]) ** 2).reshape(2 * per, -1).sum(dim=1).cpu().numpy()
    dist = torch.linalg.vector_norm((X - D["ut"]).reshape(2 * per, -1), dim=1).cpu().numpy()
    del B, X
    torch.cuda.empty_cache()
    gf, gg, L = D["gf"], D["gg"], D["L"]
    worst = 0.0
    for k, j in enumerate(js):
        df, dg = inputs.diff_direction(shape, j)
        ad = float((gf * df).sum() + sum((a * b).sum() for a, b in zip(gg, dg)))
        fd = (losses[2 * k] - losses[2 * k + 1]) / (2 * s)
        e = [stats[i].rel_residual * bnorm[i] / lam_min for i in (2 * k, 2 * k + 1)]
        err_fd = sum(2 * dist[i] * ei + ei * ei for i, ei in zip((2 * k, 2 * k + 1), e)) / (2 * s)
        err_ad = bv_norm[k] * (D["res_lam"] + 2 * D["res_u"]) / lam_min
        bound = err_fd + err_ad + 1e-14 * L / s
        worst = max(worst, abs(fd - ad) / abs(ad))
        assert abs(fd - ad) <= bound, (j, fd, ad, bound)
        # not vacuous: a 5% error (far below a dropped h^2, a flipped sign or a
        # face read one cell off) would fail
        assert bound <= 5e-2 * abs(ad), (j, bound, ad)
    print(f"diff128 chunk {chunk}: worst relative |fd - ad| / |ad| = {worst:.2e}, "
          f"sweeps {max(t.sweeps for t in stats)}")


@pytest.mark.parametrize("shape", [(20, 12, 16), (7, 9, 5)])
def test_lift_and_its_adjoint(orc, shape):
    """ms_lift against the oracle's right-hand side assembly, and
    ms_lift_adjoint as its transpose: <lift(f, g), lam> equals
    <f, grad_f> + sum_t <g_t, grad_face_t> for random f, g, lam, with each
    face gradient the slice of lam next to that face."""
    torch = torch_cuda()
    from paper_2009_12638_amd import ms
    rng = np.random.default_rng(60)
    f = rng.standard_normal(shape)
    g = inputs.random_faces(*shape, seed=61)
    lam = rng.standard_normal(shape)
    s = 0.37
    h = ms.ms_create(shape, blocks=(1, 1, 1), faces=[dev(a) for a in g])
    out = torch.empty(shape, dtype=torch.float64, device="cuda")
    say("ms_lift", shape)
    ms.ms_lift(h, dev(f), s, out)
    want = orc.lift_bc(s * f, g)
    np.testing.assert_allclose(host(out), want, rtol=2e-15, atol=0)
    gf = torch.empty(shape, dtype=torch.float64, device="cuda")
    gfaces = [torch.empty(a.shape, dtype=torch.float64, device="cuda") for a in g]
    gfaces[3] = None   # a face that is not wanted stays out
    say("ms_lift_adjoint", shape)
    ms.ms_lift_adjoint(h, dev(lam), s, gf, gfaces)
    torch.cuda.synchronize()
    np.testing.assert_array_equal(host(gf), s * lam)
    slices = [lam[0], lam[-1], lam[:, 0], lam[:, -1], lam[:, :, 0], lam[:, :, -1]]
    for t in range(6):
        if gfaces[t] is not None:
            np.testing.assert_array_equal(host(gfaces[t]), slices[t])
    lhs = float((want * lam).sum())
    rhs = float((f * host(gf)).sum()) + sum(float((g[t] * slices[t]).sum()) for t in range(6))
    assert abs(lhs - rhs) <= 1e-12 * (abs(lhs) + 1.0)
    # in place: b_eff over f
    fin = dev(f)
    ms.ms_lift(h, fin, s, fin)
    np.testing.assert_allclose(host(fin), want, rtol=2e-15, atol=0)
