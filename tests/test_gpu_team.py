"""The resident-team engine (a team of workgroups of one XCD solves one
block at a time with the block's inner vectors held in registers and LDS)
against the oracle and against the phase engine: matched synchronous sweeps
in FP64 (1e-10), mixed precision refined to tolerance (1e-6 of the FP64
oracle), overlapping blocks, boundary data, ragged and one-cell-thick blocks,
run-to-run determinism, asynchronous solves with their trace, and the
engine's refusals."""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, make, rel, say, torch_cuda

pytestmark = pytest.mark.gpu


def kappa(n):
    c = np.cos(np.pi / (n + 1))
    return (2 + 2 * c) / (2 - 2 * c)


CASES = [
    # shape, cuts, m, K, overlap
    ((64, 64, 64), [[0, 32, 64]] * 3, 10, 12, 0),
    ((48, 40, 56), [[0, 16, 48], [0, 24, 40], [0, 8, 32, 56]], 7, 9, 0),
    ((40, 36, 44), [[0, 14, 40], [0, 10, 36], [0, 20, 44]], 6, 8, 0),   # odd z cut: 2-cell vectors
    ((33, 17, 9), [[0, 11, 33], [0, 17], [0, 9]], 5, 7, 0),               # 1-cell vectors
    ((64, 64, 64), [[0, 32, 64]] * 3, 10, 10, 3),                        # overlap
    ((48, 40, 56), [[0, 16, 48], [0, 24, 40], [0, 8, 32, 56]], 8, 6, 2),
    ((6, 5, 4), [[0, 1, 2, 3, 4, 5, 6], [0, 5], [0, 2, 4]], 3, 5, 0),    # one-cell-thick blocks
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_team_matched_sweeps_fp64(orc, case):
    torch = torch_cuda()
    shape, cuts, m, K, ov = CASES[case]
    b = inputs.poisson_randn(shape, 500 + case)
    faces = inputs.random_faces(*shape, seed=520 + case)
    h, _ = make(ms, shape, cuts, faces)
    if ov:
        ms.ms_set_overlap(h, ov)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("team matched sweeps", shape, "overlap", ov)
    st = ms.ms_solve(h, dev(b), x, 0.0, m, "sync", max_sweeps=K, engine="team", history=K + 1)
    assert st.status == 0 and st.sweeps == K and st.engine == "team"
    beff = orc.lift_bc(b, faces)
    _, xo, sw, _, hist = orc.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=m, overlap=ov,
                                        max_sweeps=K)
    e = rel(host(x), xo)
    assert e <= 1e-10, e
    np.testing.assert_allclose(st.history, hist, rtol=0, atol=1e-12)
    # the phase engine gives the same iterate to rounding
    xp = torch.zeros_like(x)
    sp = ms.ms_solve(h, dev(b), xp, 0.0, m, "sync", max_sweeps=K, engine="phase")
    assert sp.engine == "phase"
    assert rel(host(x), host(xp)) <= 1e-12
    print(f"team {shape} overlap {ov}: {e:.2e} to the oracle")


@pytest.mark.parametrize("ov", [0, 2])
def test_team_mixed_to_tolerance(orc, ov):
    torch = torch_cuda()
    shape = (64, 64, 64)
    cuts = [inputs.uniform_cuts(64, 2)] * 3
    b = inputs.poisson_randn(shape, 530)
    h, _ = make(ms, shape, cuts, [None] * 6)
    if ov:
        ms.ms_set_overlap(h, ov)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("team mixed to 1e-8, overlap", ov)
    st = ms.ms_solve(h, dev(b), x, 1e-8, 10, "sync", precision="mixed", engine="team")
    assert st.status == 0
    beff = orc.lift_bc(b, [None] * 6)
    assert orc.residual(beff, host(x)) / np.linalg.norm(beff) <= 1e-8 * (1 + 1e-9)
    _, xo, sw, _, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=1e-8, m=10, overlap=ov)
    e = rel(host(x), xo)
    assert e <= 1e-6, e
    print(f"team mixed overlap {ov}: {st.sweeps} sweeps (oracle {sw}), {e:.2e}")


def test_team_inner_tol_and_determinism(orc):
    torch = torch_cuda()
    shape = (48, 48, 48)
    cuts = [inputs.uniform_cuts(48, 3)] * 3
    b = inputs.poisson_randn(shape, 531)
    h, _ = make(ms, shape, cuts, [None] * 6)
    xs = []
    for rep in range(2):
        x = torch.zeros(shape, dtype=torch.float64, device="cuda")
        say("team inner tol, run", rep)
        ms.ms_solve(h, dev(b), x, 0.0, 40, "sync", max_sweeps=6, inner_tol=0.05, engine="team")
        xs.append(x)
    assert torch.equal(xs[0], xs[1])
    beff = orc.lift_bc(b, [None] * 6)
    _, xo, _, _, _ = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=40, inner_tol=0.05,
                                      max_sweeps=6)
    assert rel(host(xs[0]), xo) <= 1e-10


def test_team_async_trace_and_bound(orc):
    torch = torch_cuda()
    n, g = 64, 4
    shape = (n, n, n)
    cuts = [inputs.uniform_cuts(n, g)] * 3
    b = inputs.poisson_randn(shape, 532)
    h, _ = make(ms, shape, cuts, [None] * 6)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    cap = 200000
    trace = torch.full((cap, 8), -7, dtype=torch.int32, device="cuda")
    say("team async with trace")
    st = ms.ms_solve(h, dev(b), x, 1e-8, 10, "async", staleness=2, engine="team", trace=trace,
                     slow_block=21, slow_sleep=200)
    assert st.status == 0 and st.engine == "team"
    rec = trace[: st.trace_len].cpu().numpy().astype(np.int64)
    bs = np.asarray(st.block_sweeps)
    assert bs.sum() == st.trace_len
    for blk in range(g ** 3):
        assert np.array_equal(np.sort(rec[rec[:, 0] == blk, 1]), np.arange(bs[blk]))
    seen = rec[:, 2:]
    gap = np.where(seen >= 0, rec[:, 1:2] - seen, -10)
    assert gap.max() <= 1 and st.max_staleness_seen == 1
    beff = orc.lift_bc(b, [None] * 6)
    assert orc.residual(beff, host(x)) / np.linalg.norm(beff) <= 1e-8 * (1 + 1e-9)
    _, xstar, _, _ = orc.cg(beff, np.zeros(shape), tol=1e-13, max_iters=20000)
    assert rel(host(x), xstar) <= kappa(n) * 1e-8
    print(f"team async: sweeps per block {bs.min()}..{bs.max()}, relaunches {st.relaunches}")


def test_team_refusals():
    torch = torch_cuda()
    # one 512^2 x 16 block does not fit a team (slab of 16 planes x 512^2 cells)
    shape = (16, 512, 512)
    h = ms.ms_create(shape, blocks=(1, 1, 1))
    b = torch.zeros(shape, dtype=torch.float64, device="cuda")
    b[3, 4, 5] = 1.0
    x = torch.zeros_like(b)
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve(h, b, x, 1e-6, 5, "sync", engine="team", max_sweeps=3)
    assert e.value.status == ms.MS_ERR_UNSUPPORTED
    # auto falls back to the phase engine
    st = ms.ms_solve(h, b, x, 0.0, 5, "sync", max_sweeps=2)
    assert st.status == 0 and st.engine == "phase"
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve(h, b, x, 1e-6, 5, "sync", engine=7)
    assert e.value.status == ms.MS_ERR_ARG


@pytest.mark.parametrize("mode", ["sync", "async"])
def test_team_bounded_waits_fail_cleanly(orc, mode):
    """A team-engine wait that gives up (forced from the host with a spin
    limit of one poll: the launch's start or a team barrier cannot complete
    in time) ends every workgroup, fails the solve with MS_ERR_HIP and leaves
    the handle usable: the next solve on it matches the oracle."""
    torch = torch_cuda()
    n, g = 48, 3
    shape = (n, n, n)
    cuts = [inputs.uniform_cuts(n, g)] * 3
    b = inputs.poisson_randn(shape, 540)
    h, _ = make(ms, shape, cuts, [None] * 6)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("team forced wait failure", mode)
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve(h, dev(b), x, 1e-8, 10, mode, engine="team", team_spin=1, max_sweeps=50)
    assert e.value.status == ms.MS_ERR_HIP
    assert "team engine" in str(e.value)
    with pytest.raises(ms.MsError) as e:
        ms.ms_solve(h, dev(b), x, 1e-8, 10, mode, engine="team", team_spin=-1)
    assert e.value.status == ms.MS_ERR_ARG
    x.zero_()
    st = ms.ms_solve(h, dev(b), x, 1e-8, 10, mode, engine="team")
    assert st.status == 0 and st.engine == "team"
    beff = orc.lift_bc(b, [None] * 6)
    assert orc.residual(beff, host(x)) / np.linalg.norm(beff) <= 1e-8 * (1 + 1e-9)
    if mode == "sync":
        _, xo, sw, _, _ = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-8, m=10)
        assert sw == st.sweeps
        assert rel(host(x), xo) <= 1e-10
    print(f"team {mode}: forced wait failure reported, next solve {st.sweeps} sweeps")
