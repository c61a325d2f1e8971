"""The allocation-free residual entry point (static scratch) against
ms_residual on the same inputs: two calls in a row on different handles,
the second on a smaller grid, then the size limit."""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, make, say, torch_cuda

pytestmark = pytest.mark.gpu


def one_case(orc, shape, cuts, seed, overlap=0):
    torch = torch_cuda()
    faces = inputs.random_faces(*shape, seed=seed)
    h, _ = make(ms, shape, cuts, faces)
    if overlap:
        ms.ms_set_overlap(h, overlap)
    bh = inputs.poisson_randn(shape, seed + 1)
    b = dev(bh)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    ms.ms_solve(h, b, x, 0.0, 5, "sync", max_sweeps=3)
    say("no-alloc residual", shape, "overlap", overlap)
    got = ms.ms_residual_noalloc(h, b, x)
    want = ms.ms_residual(h, b, x)
    # same kernels, same fixed-order sums: bitwise equal
    assert got == want, (got, want)
    beff = orc.lift_bc(bh, faces)
    xr = host(x)
    ref_abs = orc.residual(beff, xr)
    ref_rel = ref_abs / np.linalg.norm(beff)
    assert abs(got[0] - ref_rel) <= 1e-12 * ref_rel
    assert abs(got[1] - ref_abs) <= 1e-12 * ref_abs
    return got


def test_noalloc_residual_matches_ms_residual(orc):
    a = one_case(orc, (48, 40, 56), [[0, 16, 48], [0, 24, 40], [0, 8, 32, 56]], 300)
    b = one_case(orc, (20, 12, 16), [[0, 10, 20], [0, 12], [0, 16]], 302)
    c = one_case(orc, (32, 32, 32), [inputs.uniform_cuts(32, 2)] * 3, 304, overlap=2)
    assert a != b and b != c


def test_noalloc_residual_rejects_too_many_tiles():
    torch = torch_cuda()
    shape = (64, 64, 64)
    # 131072 blocks of 1x1x2 cells: one tile each, twice what the scratch holds
    h = ms.ms_create(shape, blocks=(64, 64, 32))
    b = torch.zeros(shape, dtype=torch.float64, device="cuda")
    x = torch.zeros_like(b)
    with pytest.raises(ms.MsError) as e:
        ms.ms_residual_noalloc(h, b, x)
    assert e.value.status == ms.MS_ERR_ARG and "tiles" in e.value.msg
    # the handle-scratch entry point still serves it
    assert ms.ms_residual(h, b, x) == (0.0, 0.0)
