"""The autotuner returns valid options, caches them, and the tuned options
solve the same problem to the same answer."""
import os

import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, say, torch_cuda

pytestmark = pytest.mark.gpu


def test_autotune_valid_and_cached(tmp_path, orc):
    torch = torch_cuda()
    from paper_2009_12638_amd import tune
    shape = (64, 64, 64)
    cuts = [inputs.uniform_cuts(64, 2)] * 3
    b = dev(inputs.poisson_randn(shape, 140))
    cache = str(tmp_path / "tune.json")
    say("autotune 64^3")
    out = tune.autotune(shape, cuts, b, precision="mixed", cache=cache)
    assert out["rows"] in (1, 2, 4) and out["x_chunk"] in (8, 16, 32)
    assert out["inner_iters"] in tune.INNER_CANDIDATES
    assert out["group_blocks"] in tune.GROUP_CANDIDATES
    assert os.path.exists(cache)
    again = tune.autotune(shape, cuts, b, precision="mixed", cache=cache)
    assert again == out
    # tuned tiling changes the schedule, not the arithmetic: same iterate as default
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts])
    x1 = torch.zeros(shape, dtype=torch.float64, device="cuda")
    x2 = torch.zeros_like(x1)
    ms.ms_solve(h, b, x1, 0.0, 10, "sync", max_sweeps=6, precision="mixed")
    ms.ms_solve(h, b, x2, 0.0, 10, "sync", max_sweeps=6, precision="mixed",
                rows=out["rows"], x_chunk=out["x_chunk"], group_blocks=out["group_blocks"])
    d = float(torch.linalg.norm(x1 - x2) / torch.linalg.norm(x1))
    assert d <= 1e-5   # FP32 inner sums in a different tile order


def _replay(orc, beff, cuts, schedule, tol):
    """The oracle run through the same (m, sweeps) schedule, warm-starting
    each piece from the previous iterate."""
    x = np.zeros(beff.shape)
    total = 0
    for m, n in schedule:
        st, x, sw, _, _ = orc.block_jacobi(beff, x, cuts, tol=tol, m=m, max_sweeps=n)
        total += sw
        if st == 0:
            break
    return st, x, total


def test_scheduled_inner_iterations_match_oracle(orc):
    """Inner-iteration counts that change with the outer iteration (an
    explicit schedule): the same iterate and sweep count as the oracle run
    through the same schedule."""
    torch = torch_cuda()
    from paper_2009_12638_amd import tune
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    b = inputs.poisson_randn(shape, 141)
    beff = orc.lift_bc(b, [None] * 6)
    h = ms.ms_create(shape, cuts=[list(c) for c in cuts])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    schedule = [(3, 40), (12, 25), (6, 10**6)]
    say("scheduled inner iterations")
    st, total, res = tune.solve_schedule(h, dev(b), x, 1e-8, schedule)
    ms.ms_destroy(h)
    ost, xo, ototal = _replay(orc, beff, cuts, schedule, 1e-8)
    assert st == 0 and ost == 0 and total == ototal and res <= 1e-8
    assert float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)) <= 1e-10


def test_adaptive_inner_iterations_replay(orc):
    """The adaptive solve reaches tol, changes m along the way, and its
    recorded schedule replayed by the oracle gives the same iterate."""
    torch = torch_cuda()
    from paper_2009_12638_amd import tune
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    b = inputs.poisson_randn(shape, 142)
    beff = orc.lift_bc(b, [None] * 6)
    h = ms.ms_create(shape, cuts=[list(c) for c in cuts])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("adaptive inner iterations")
    st, total, res, schedule = tune.solve_adaptive(h, dev(b), x, 1e-8, m0=4, chunk=30)
    ms.ms_destroy(h)
    assert st == 0 and res <= 1e-8
    assert len({m for m, _ in schedule}) > 1, schedule
    ost, xo, ototal = _replay(orc, beff, cuts, schedule, 1e-8)
    assert ost == 0 and ototal == total, (ototal, total)
    assert float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)) <= 1e-10


def test_tune_overlap_and_inner(orc):
    """The (overlap, m) tuner solves a proxy with the same block shapes for
    every pair; with the real problem given it times each pair's sweep there
    and returns the pair with the smallest proxy sweeps x real sweep time;
    the proxy keeps the block shapes; a solve of the real problem with the
    chosen pair matches the oracle's overlapping block Jacobi with the same
    m."""
    torch = torch_cuda()
    from paper_2009_12638_amd import tune
    shape, cuts = (48, 40, 36), ([0, 16, 32, 48], [0, 20, 40], [0, 12, 24, 36])
    pshape, pcuts, _ = tune.proxy_problem(shape, cuts)
    assert pshape == (32, 40, 24) and pcuts == [[0, 16, 32], [0, 20, 40], [0, 12, 24]]
    say("tune overlap and m")
    best, results = tune.tune_overlap_inner(shape, cuts, precision="mixed", overlaps=(0, 2),
                                            inners=(5, 10), tol=1e-6)
    assert len(results) == 4 and best in results and best["converged"]
    assert best["seconds"] == min(r["seconds"] for r in results if r["converged"])
    b = inputs.poisson_randn(shape, 143)
    h = ms.ms_create(shape, cuts=[list(c) for c in cuts])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("tune overlap and m, real sweep times")
    best, results = tune.tune_overlap_inner(shape, cuts, precision="mixed", overlaps=(0, 2),
                                            inners=(5, 10), tol=1e-6, full=(h, dev(b), x))
    done = [r for r in results if r["converged"]]
    assert best in done and all(r["full_ms_per_sweep"] > 0 for r in done)
    assert best["estimate"] == min(r["estimate"] for r in done)
    for r in done:
        assert r["estimate"] == pytest.approx(r["sweeps"] * r["full_ms_per_sweep"] / 1e3)
    ms.ms_set_overlap(h, best["overlap"])
    x.zero_()
    st = ms.ms_solve(h, dev(b), x, 1e-8, best["m"], "sync")
    ms.ms_destroy(h)
    beff = orc.lift_bc(b, [None] * 6)
    ost, xo, K, _, _ = orc.multisplit(beff, np.zeros(shape), cuts, tol=1e-8, m=best["m"],
                                      overlap=best["overlap"])
    assert st.status == 0 and ost == 0 and st.sweeps == K
    assert float(np.linalg.norm(host(x) - xo) / np.linalg.norm(xo)) <= 1e-10
