"""Parity at full size, in the launch configuration the benchmark times.

A synchronous sweep updates each block from the previous iterate only
(Section 3: X_i^(k) from sweep k-1 values), so one GPU sweep can be checked
block by block: from the GPU's own iterate x^(2) the oracle recomputes the
new values of a few sampled blocks (a corner, edges, interior ones) and they
are compared with the GPU's x^(3) on those blocks.
"""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

# Tolerance on the block correction d = x^(3) - x^(2): FP64 differs only by
# summation order (observed ~1e-14); FP32 inner CG differs from the FP64
# oracle by FP32 rounding amplified by at most the block condition number
# (about 1.7e3 for a 64^3 block, so ~1e-4), hence 1e-3.
D_TOL = {"fp64": 1e-10, "mixed": 1e-3}

_cache = {}


def workload(name):
    if name not in _cache:
        _cache.clear()
        _cache[name] = inputs.workload(name)
    return _cache[name]


def sampled_blocks(g):
    """corner, opposite corner, an edge block and two interior blocks"""
    def num(i, j, k):
        return (i * g + j) * g + k
    picks = {num(0, 0, 0), num(g - 1, g - 1, g - 1), num(0, g // 2, g - 1),
             num(g // 2, g // 2, g // 2), num(g - 2, 1, g // 2 - 1)}
    return sorted(picks)


@pytest.mark.parametrize("name,precision,ov", [("poisson256", "fp64", 0), ("bumps512", "fp64", 0),
                                               ("bumps512", "mixed", 0), ("bumps512", "fp64", 1),
                                               ("bumps512", "mixed", 4)])
def test_sampled_block_sweep(orc, name, precision, ov):
    """ov > 0: overlapping blocks (regions of depth ov); the oracle's
    per-block sweep then solves on each sampled block's region."""
    torch = torch_cuda()
    w = workload(name)
    shape, cuts = w["shape"], w["cuts"]
    g = len(cuts[0]) - 1
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    if ov:
        ms.ms_set_overlap(h, ov)
    b = dev(w["b"])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("fullsize", name, precision, "overlap", ov, "2 sweeps")
    ms.ms_solve(h, b, x, 0.0, w["m"], "sync", max_sweeps=2, precision=precision)
    x2 = host(x)
    say("fullsize", name, precision, "1 more sweep")
    ms.ms_solve(h, b, x, 0.0, w["m"], "sync", max_sweeps=1, precision=precision)
    x3 = host(x)
    del x, b
    ms.ms_destroy(h)
    torch.cuda.empty_cache()
    beff = orc.lift_bc(w["b"], [None] * 6)
    blocks = sampled_blocks(g)
    if ov:
        xo = orc.ovl_sweep_some(beff, x2, cuts, ov, blocks, m=w["m"])
    else:
        xo = orc.block_sweep_some(beff, x2, cuts, blocks, m=w["m"])
    cx, cy, cz = cuts
    worst = 0.0
    for blk in blocks:
        bi, bj, bk = blk // (g * g), (blk // g) % g, blk % g
        sl = (slice(cx[bi], cx[bi + 1]), slice(cy[bj], cy[bj + 1]), slice(cz[bk], cz[bk + 1]))
        d_gpu = x3[sl] - x2[sl]
        d_or = xo[sl] - x2[sl]
        e = rel(d_gpu, d_or)
        worst = max(worst, e)
        assert e <= D_TOL[precision], (blk, e)
    # every other block moved too (nothing skipped), and nothing is non-finite
    assert np.isfinite(x3).all()
    moved = np.abs(x3 - x2).reshape(g, shape[0] // g, g, shape[1] // g, g, shape[2] // g)
    assert (moved.max(axis=(1, 3, 5)) > 0).all()
    print(f"{name} {precision} overlap {ov}: worst block correction error {worst:.2e}")


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_bumps512_gmres_sampled_blocks(orc, precision):
    """GMRES(10) inner solves at 512^3 (the paper's inner solver): one GPU
    sweep from the GPU's own iterate against the oracle's per-block GMRES
    sweep on sampled blocks."""
    torch = torch_cuda()
    w = workload("bumps512")
    shape, cuts = w["shape"], w["cuts"]
    g = len(cuts[0]) - 1
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    ms.ms_reserve_krylov(h, w["m"])
    b = dev(w["b"])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("fullsize gmres", precision, "2 sweeps")
    ms.ms_solve(h, b, x, 0.0, w["m"], "sync", max_sweeps=2, precision=precision, inner="gmres")
    x2 = host(x)
    say("fullsize gmres", precision, "1 more sweep")
    ms.ms_solve(h, b, x, 0.0, w["m"], "sync", max_sweeps=1, precision=precision, inner="gmres")
    x3 = host(x)
    del x, b
    ms.ms_destroy(h)
    torch.cuda.empty_cache()
    beff = orc.lift_bc(w["b"], [None] * 6)
    blocks = sampled_blocks(g)
    xo = orc.multisplit_sweep_some(beff, x2, cuts, blocks, m=w["m"], inner="gmres")
    cx, cy, cz = cuts
    worst = 0.0
    for blk in blocks:
        bi, bj, bk = blk // (g * g), (blk // g) % g, blk % g
        sl = (slice(cx[bi], cx[bi + 1]), slice(cy[bj], cy[bj + 1]), slice(cz[bk], cz[bk + 1]))
        e = rel(x3[sl] - x2[sl], xo[sl] - x2[sl])
        worst = max(worst, e)
        assert e <= D_TOL[precision], (blk, e)
    assert np.isfinite(x3).all()
    print(f"bumps512 gmres {precision}: worst block correction error {worst:.2e}")


def test_uneven384_batch_sampled_blocks(orc):
    """The batched workload at full size (384x320x448, uneven blocks with
    edges from {32,48,64,96}, 16 right-hand sides, mixed precision): sampled
    blocks of sampled right-hand sides against the oracle's block sweep."""
    torch = torch_cuda()
    w = workload("uneven384")
    shape, cuts = w["shape"], w["cuts"]
    nrhs = w["b"].shape[0]
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    ms.ms_reserve(h, nrhs)
    B = torch.from_numpy(w["b"]).to("cuda")
    X = torch.zeros_like(B)
    say("uneven384 batch 2 sweeps")
    ms.ms_solve_batch(h, B, X, 0.0, w["m"], max_sweeps=2, precision="mixed")
    picks = [0, 7, nrhs - 1]
    x2 = {k: host(X[k]) for k in picks}
    say("uneven384 batch 1 more sweep")
    ms.ms_solve_batch(h, B, X, 0.0, w["m"], max_sweeps=1, precision="mixed")
    x3 = {k: host(X[k]) for k in picks}
    del X, B
    ms.ms_destroy(h)
    torch.cuda.empty_cache()
    gx, gy, gz = (len(c) - 1 for c in cuts)
    blocks = sorted({0, gx * gy * gz - 1, (gx // 2 * gy + gy // 2) * gz + gz // 2,
                     (1 * gy + 0) * gz + gz - 2})
    worst = 0.0
    for k in picks:
        beff = orc.lift_bc(w["b"][k], [None] * 6)
        xo = orc.block_sweep_some(beff, x2[k], cuts, blocks, m=w["m"])
        for blk in blocks:
            bi, bj, bk = blk // (gy * gz), (blk // gz) % gy, blk % gz
            sl = (slice(cuts[0][bi], cuts[0][bi + 1]), slice(cuts[1][bj], cuts[1][bj + 1]),
                  slice(cuts[2][bk], cuts[2][bk + 1]))
            e = rel(x3[k][sl] - x2[k][sl], xo[sl] - x2[k][sl])
            worst = max(worst, e)
            assert e <= D_TOL["mixed"], (k, blk, e)
    print(f"uneven384 batch: worst block correction error {worst:.2e}")
