"""GPU checks of the asynchronous sweep (Sections 2.1 and 2.3: blocks use
the latest neighbour values they have) and of the global CG baseline.

Asynchronous iterates depend on timing, so they are checked by what must
hold whatever the interleaving: the verified FP64 residual meets tol, the
distance to the exact solution is within kappa * tol, the staleness bound is
never exceeded, and fixed-sweep runs do exactly the requested work.  The
global CG is compared with the oracle's CG iterate by iterate."""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, make, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def kappa(n):
    """condition number of the 7-point operator on an n^3 grid (closed form)"""
    c = np.cos(np.pi / (n + 1))
    return (2 + 2 * c) / (2 - 2 * c)


@pytest.fixture(scope="module")
def laplace32(orc):
    w = inputs.workload("laplace32")
    beff = orc.lift_bc(w["b"], w["faces"])
    _, xstar, _, _, _ = orc.block_jacobi(beff, np.zeros(w["shape"]), w["cuts"], tol=1e-13, m=20)
    return w, xstar


@pytest.mark.parametrize("S,precision", [(1, "fp64"), (2, "fp64"), (4, "fp64"), (2, "mixed")])
def test_async_converges_within_kappa_bound(laplace32, S, precision):
    torch = torch_cuda()
    w, xstar = laplace32
    h, _ = make(ms, w["shape"], w["cuts"], w["faces"])
    x = torch.zeros(w["shape"], dtype=torch.float64, device="cuda")
    say("async laplace32 S", S, precision)
    st = ms.ms_solve(h, dev(w["b"]), x, 1e-8, 10, "async", staleness=S, precision=precision,
                     history=64)
    assert st.status == 0
    assert st.rel_residual <= 1e-8
    relr, _ = ms.ms_residual(h, dev(w["b"]), x)
    assert relr <= 1e-8
    assert rel(host(x), xstar) <= kappa(32) * 1e-8
    assert 0 <= st.max_staleness_seen <= S - 1
    print(f"async S={S} {precision}: ~{st.sweeps} sweeps/block, staleness {st.max_staleness_seen},"
          f" relaunches {st.relaunches}")


@pytest.mark.parametrize("shape,cuts", [
    ((40, 36, 44), ([0, 14, 40], [0, 10, 36], [0, 20, 44])),
    ((64, 64, 64), ([0, 32, 64], [0, 32, 64], [0, 32, 64])),
])
def test_async_fixed_sweeps_do_the_requested_work(orc, shape, cuts):
    """tol <= 0: every block runs exactly max_sweeps sweeps of m iterations,
    and the result is a valid iterate that improved the residual."""
    torch = torch_cuda()
    rng = np.random.default_rng(200)
    b = rng.standard_normal(shape) / 100
    faces = inputs.random_faces(*shape, seed=201)
    h, _ = make(ms, shape, cuts, faces)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    K, m = 12, 6
    say("async fixed sweeps", shape)
    st = ms.ms_solve(h, dev(b), x, 0.0, m, "async", max_sweeps=K, staleness=2)
    nb = (len(cuts[0]) - 1) * (len(cuts[1]) - 1) * (len(cuts[2]) - 1)
    assert st.status == 0 and st.sweeps == K
    assert st.inner_iters == K * nb * m
    assert st.max_staleness_seen <= 1
    beff = orc.lift_bc(b, faces)
    r0 = np.linalg.norm(beff)
    assert orc.residual(beff, host(x)) < 0.5 * r0
    # the synchronous method after the same number of sweeps is of the same quality
    _, xs, _, _, hs = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=m, max_sweeps=K)
    assert orc.residual(beff, host(x)) / r0 < 100 * hs[-1]


def test_async_uneven_blocks_reach_tolerance(orc):
    torch = torch_cuda()
    shape = (48, 40, 56)
    cuts = ([0, 16, 48], [0, 24, 40], [0, 8, 32, 56])
    b = inputs.poisson_randn(shape, 202)
    h, _ = make(ms, shape, cuts, [None] * 6)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("async uneven")
    st = ms.ms_solve(h, dev(b), x, 1e-9, 8, "async", staleness=3)
    assert st.status == 0 and st.rel_residual <= 1e-9
    beff = orc.lift_bc(b, [None] * 6)
    _, xstar, _, _, _ = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-13, m=20)
    assert rel(host(x), xstar) <= kappa(max(shape)) * 1e-9
    assert st.max_staleness_seen <= 2


def test_async_not_converged_and_zero_rhs():
    torch = torch_cuda()
    shape = (32, 32, 32)
    h, _ = make(ms, shape, [inputs.uniform_cuts(32, 2)] * 3, [None] * 6)
    b = dev(inputs.poisson_randn(shape, 203))
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("async not converged")
    st = ms.ms_solve(h, b, x, 1e-14, 5, "async", max_sweeps=4, raise_on_error=False)
    assert st.status == ms.MS_ERR_NOT_CONVERGED and st.sweeps == 4
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve(h, b, x, 1e-8, 5, "async", staleness=0)
    assert e.value.status == ms.MS_ERR_ARG
    z = torch.zeros_like(b)
    x.fill_(1.0)
    st = ms.ms_solve(h, z, x, 1e-8, 5, "async")
    assert not host(x).any()


# ----------------------------------------------------------------------
# global CG baseline
# ----------------------------------------------------------------------

@pytest.mark.parametrize("shape", [(24, 20, 28), (17, 9, 13)])
def test_global_cg_matches_oracle_iterates(orc, shape):
    torch = torch_cuda()
    rng = np.random.default_rng(204)
    b = rng.standard_normal(shape)
    faces = inputs.random_faces(*shape, seed=205)
    h, _ = make(ms, shape, [[0, shape[0]], [0, shape[1]], [0, shape[2]]], faces)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    K = 25
    say("global cg", shape)
    st = ms.ms_cg(h, dev(b), x, 0.0, K, history=K + 1)
    beff = orc.lift_bc(b, faces)
    ost, xo, it, hist = orc.cg(beff, np.zeros(shape), tol=0.0, max_iters=K)
    assert st.status == 0 and st.sweeps == K == it
    assert rel(host(x), xo) <= 1e-10, rel(host(x), xo)
    np.testing.assert_allclose(st.history, hist, rtol=1e-9, atol=1e-13)


def test_global_cg_to_tolerance(orc):
    torch = torch_cuda()
    w = inputs.workload("laplace32")
    beff = orc.lift_bc(w["b"], w["faces"])
    ost, xo, it, hist = orc.cg(beff, np.zeros(w["shape"]), tol=1e-8, max_iters=2000)
    h, _ = make(ms, w["shape"], w["cuts"], w["faces"])
    x = torch.zeros(w["shape"], dtype=torch.float64, device="cuda")
    say("global cg laplace32")
    st = ms.ms_cg(h, dev(w["b"]), x, 1e-8, 2000)
    assert st.status == 0 and abs(st.sweeps - it) <= 1
    # reported residual is the true one (recurrence and true agree to ~1e-14 here)
    assert st.rel_residual <= 1.01e-8
    assert rel(host(x), xo) <= 1e-9
