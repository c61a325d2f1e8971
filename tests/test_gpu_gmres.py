"""GPU parity of GMRES inner solves (Sections 3.1 and 4: the paper's inner
Krylov solver) through the C ABI against the CPU oracle's GMRES(m) cycle:
FP64 iterates after the same number of sweeps to 1e-10 (with and without
overlap, ragged blocks, several right-hand sides), mixed precision to the
FP64 answer within 1e-6, and the error paths."""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, make, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

TOL_FP64 = 1e-10
TOL_MIXED = 1e-6
HIST_ATOL = 1e-12


def _gpu(shape, cuts, b, faces, ov, m, K, precision="fp64", reserve=None, **kw):
    torch = torch_cuda()
    h, _ = make(ms, shape, cuts, faces)
    if ov:
        ms.ms_set_overlap(h, ov)
    ms.ms_reserve_krylov(h, reserve or m)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("gmres solve", shape, "o", ov, "m", m, "K", K, precision, kw)
    st = ms.ms_solve(h, dev(b), x, 0.0, m, "sync", max_sweeps=K, precision=precision,
                     history=K + 1, inner="gmres", **kw)
    ms.ms_destroy(h)
    return st, host(x)


CASES = [
    # shape, cuts, overlap, m, K
    ((40, 36, 44), ([0, 14, 40], [0, 10, 36], [0, 20, 44]), 0, 6, 12),
    ((33, 30, 26), ([0, 11, 33], [0, 16, 30], [0, 13, 26]), 0, 5, 10),   # odd z: scalar path
    ((40, 36, 44), ([0, 14, 40], [0, 10, 36], [0, 20, 44]), 2, 5, 10),   # overlap regions
    ((24, 24, 64), ([0, 24], [0, 24], [0, 64]), 0, 12, 4),              # one block
    ((8, 6, 4), ([0, 1, 2, 3, 4, 5, 6, 7, 8], [0, 2, 4, 6], [0, 2, 4]), 0, 2, 8),  # tiny blocks
]


@pytest.mark.parametrize("shape,cuts,ov,m,K", CASES)
def test_gmres_fp64_matched(orc, shape, cuts, ov, m, K):
    rng = np.random.default_rng(400 + m)
    b = rng.standard_normal(shape) / 100
    faces = inputs.random_faces(*shape, seed=401)
    st, xg = _gpu(shape, cuts, b, faces, ov, m, K)
    beff = orc.lift_bc(b, faces)
    ost, xo, sw, inner, hist = orc.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=m,
                                              overlap=ov, inner="gmres", max_sweeps=K)
    assert ost == 0 and sw == K
    assert st.status == 0 and st.sweeps == K
    assert rel(xg, xo) <= TOL_FP64, rel(xg, xo)
    assert st.inner_iters == inner, (st.inner_iters, inner)
    np.testing.assert_allclose(st.history, hist, rtol=1e-9, atol=HIST_ATOL)


def test_gmres_inner_tol_matches_oracle(orc):
    shape, cuts = (40, 36, 44), ([0, 14, 40], [0, 10, 36], [0, 20, 44])
    rng = np.random.default_rng(402)
    b = rng.standard_normal(shape) / 100
    st, xg = _gpu(shape, cuts, b, [None] * 6, 0, 20, 8, inner_tol=1e-2)
    beff = orc.lift_bc(b, [None] * 6)
    _, xo, _, inner, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=20,
                                        inner="gmres", inner_tol=1e-2, max_sweeps=8)
    assert rel(xg, xo) <= TOL_FP64
    assert st.inner_iters == inner
    assert inner < 8 * 8 * 20      # the inner tolerance stopped some cycles early


def test_gmres_to_tolerance(orc):
    """The GPU's stopping rule with GMRES inner solves stops where the
    oracle's does; the reserved basis may be larger than m."""
    torch = torch_cuda()
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    b = inputs.poisson_randn(shape, 403)
    beff = orc.lift_bc(b, [None] * 6)
    ost, xo, K, _, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=1e-8, m=8, inner="gmres")
    assert ost == 0
    h, _ = make(ms, shape, cuts, [None] * 6)
    ms.ms_reserve_krylov(h, 16)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("gmres to tol")
    st = ms.ms_solve(h, dev(b), x, 1e-8, 8, "sync", inner="gmres")
    ms.ms_destroy(h)
    assert st.status == 0 and st.sweeps == K and st.rel_residual <= 1e-8
    assert rel(host(x), xo) <= TOL_FP64


@pytest.mark.parametrize("ov", [0, 4])
def test_gmres_mixed_refines_to_fp64(orc, ov):
    torch = torch_cuda()
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    b = inputs.poisson_randn(shape, 404)
    faces = inputs.random_faces(*shape, seed=405)
    beff = orc.lift_bc(b, faces)
    ost, xo, K, _, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=1e-8, m=8, overlap=ov,
                                      inner="gmres")
    h, _ = make(ms, shape, cuts, faces)
    if ov:
        ms.ms_set_overlap(h, ov)
    ms.ms_reserve_krylov(h, 8)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("gmres mixed", ov)
    st = ms.ms_solve(h, dev(b), x, 1e-8, 8, "sync", precision="mixed", inner="gmres")
    ms.ms_destroy(h)
    assert st.status == 0 and st.rel_residual <= 1e-8
    assert rel(host(x), xo) <= TOL_MIXED, rel(host(x), xo)
    assert abs(st.sweeps - K) <= max(3, K // 20), (st.sweeps, K)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_gmres_batch_and_graph(precision):
    """Several right-hand sides in the same launches equal single solves, and
    graph replay equals eager launches, bit for bit."""
    torch = torch_cuda()
    shape, cuts = (32, 24, 48), ([0, 8, 16, 32], [0, 12, 24], [0, 16, 32, 48])
    rng = np.random.default_rng(406)
    B = dev(rng.standard_normal((3,) + shape))
    h, _ = make(ms, shape, cuts, [None] * 6)
    ms.ms_reserve(h, 3)
    ms.ms_reserve_krylov(h, 6)
    X = torch.zeros_like(B)
    say("gmres batch", precision)
    ms.ms_solve_batch(h, B, X, 0.0, 6, max_sweeps=9, precision=precision, inner="gmres")
    for k in range(3):
        x = torch.zeros(shape, dtype=torch.float64, device="cuda")
        ms.ms_solve(h, B[k].contiguous(), x, 0.0, 6, "sync", max_sweeps=9, precision=precision,
                    inner="gmres")
        assert torch.equal(x, X[k]), k
        xe = torch.zeros_like(x)
        ms.ms_solve(h, B[k].contiguous(), xe, 0.0, 6, "sync", max_sweeps=9, precision=precision,
                    inner="gmres", use_graph=False)
        assert torch.equal(x, xe), k
    ms.ms_destroy(h)


def test_gmres_errors():
    torch = torch_cuda()
    shape = (16, 16, 16)
    h, _ = make(ms, shape, [inputs.uniform_cuts(16, 2)] * 3, [None] * 6)
    b = torch.ones(shape, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(ms.MsError) as e:          # no basis reserved
        ms.ms_solve(h, b, x, 1e-6, 5, "sync", inner="gmres")
    assert e.value.status == ms.MS_ERR_ARG
    ms.ms_reserve_krylov(h, 4)
    with pytest.raises(ms.MsError) as e:          # m above the reserved basis
        ms.ms_solve(h, b, x, 1e-6, 5, "sync", inner="gmres")
    assert e.value.status == ms.MS_ERR_ARG
    with pytest.raises(ms.MsError) as e:
        ms.ms_reserve_krylov(h, 0)
    assert e.value.status == ms.MS_ERR_ARG
    ms.ms_reserve(h, 2)                           # the basis must follow the new capacity
    B = torch.ones((2,) + shape, dtype=torch.float64, device="cuda")
    X = torch.zeros_like(B)
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve_batch(h, B, X, 1e-6, 4, inner="gmres")
    assert e.value.status == ms.MS_ERR_ARG
    ms.ms_reserve_krylov(h, 4)
    st = ms.ms_solve_batch(h, B, X, 1e-6, 4, inner="gmres")
    assert all(s.status == 0 for s in st)
    ms.ms_destroy(h)


def _kappa(shape):
    lo = sum(2 - 2 * np.cos(np.pi / (n + 1)) for n in shape)
    hi = sum(2 + 2 * np.cos(np.pi / (n + 1)) for n in shape)
    return hi / lo


def test_gmres_async_single_block_matches_oracle(orc):
    """One block: the asynchronous worker runs GMRES(m) cycles on the whole
    grid one after another, which is the synchronous method exactly; FP64
    iterates after K sweeps match the oracle to 1e-10."""
    torch = torch_cuda()
    shape, cuts = (24, 20, 32), ([0, 24], [0, 20], [0, 32])
    rng = np.random.default_rng(407)
    b = rng.standard_normal(shape) / 100
    faces = inputs.random_faces(*shape, seed=408)
    h, _ = make(ms, shape, cuts, faces)
    ms.ms_reserve_krylov(h, 7)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("gmres async one block")
    st = ms.ms_solve(h, dev(b), x, 0.0, 7, "async", max_sweeps=6, inner="gmres")
    ms.ms_destroy(h)
    beff = orc.lift_bc(b, faces)
    _, xo, _, inner, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=7,
                                        inner="gmres", max_sweeps=6)
    assert st.status == 0 and st.inner_iters == inner
    assert rel(host(x), xo) <= TOL_FP64, rel(host(x), xo)


@pytest.mark.parametrize("ov,S,precision", [(0, 2, "fp64"), (2, 1, "fp64"), (0, 2, "mixed"),
                                            (4, 2, "mixed")])
def test_gmres_async_converges(orc, ov, S, precision):
    """Asynchronous sweeps with GMRES inner solves (the paper's configuration),
    with and without overlap: verified residual, kappa bound to the exact
    solution, staleness bound."""
    torch = torch_cuda()
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    b = inputs.poisson_randn(shape, 409)
    faces = inputs.random_faces(*shape, seed=410)
    beff = orc.lift_bc(b, faces)
    _, xstar, _, _ = orc.cg(beff, np.zeros(shape), tol=1e-14, max_iters=5000)
    h, _ = make(ms, shape, cuts, faces)
    if ov:
        ms.ms_set_overlap(h, ov)
    ms.ms_reserve_krylov(h, 8)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("gmres async", ov, S, precision)
    st = ms.ms_solve(h, dev(b), x, 1e-8, 8, "async", staleness=S, precision=precision,
                     inner="gmres")
    relr, _ = ms.ms_residual(h, dev(b), x)
    ms.ms_destroy(h)
    assert st.status == 0 and st.rel_residual <= 1e-8 and relr <= 1e-8
    assert rel(host(x), xstar) <= _kappa(shape) * 1e-8
    assert 0 <= st.max_staleness_seen <= S - 1 and st.inner_iters > 0
    print(f"gmres async o={ov} S={S} {precision}: ~{st.sweeps} sweeps/block, "
          f"staleness {st.max_staleness_seen}, relaunches {st.relaunches}")
