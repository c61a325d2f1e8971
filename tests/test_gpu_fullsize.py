"""Parity at full size, in the launch configuration the benchmark times.

Whole grids: the GPU's iterate after K synchronous sweeps against the
oracle's after the same K sweeps (FP64 to 1e-10 relative L2, at 256^3 with
K = 50 and at 512^3 with K = 8; mixed precision at 512^3 against the FP64
oracle), and a mixed-precision solve to 1e-8 against the FP64 oracle's
solve to 1e-8 (1e-6, at 128^3).

Sampled blocks: a synchronous sweep updates each block from the previous
iterate only (Section 3: X_i^(k) from sweep k-1 values), so one GPU sweep
can be checked block by block: from the GPU's own iterate x^(2) the oracle
recomputes the new values of a few sampled blocks (a corner, edges,
interior ones) and they are compared with the GPU's x^(3) on those blocks.
"""
import numpy as np
import pytest

from paper_2009_12638_amd import inputs, ms
from gpu_util import dev, host, rel, say, torch_cuda

pytestmark = pytest.mark.gpu

# Tolerance on the block correction d = x^(3) - x^(2).  FP64 differs only by
# summation order (observed ~1e-14).  Mixed: the FP32 inner CG starts from
# the residual rounded to FP32 (relative u/2, u = 2^-24 = 6e-8) and each of
# its m = 10 steps rounds the updated d once more (relative u); alpha and
# beta carry the rounding of the dot products, but CG corrects a perturbed
# step size in its next steps to first order, so the correction is off by
# about (m + 1) u = 6.6e-7 (observed 2-4e-7).  The bar allows 3x that.
D_TOL = {"fp64": 1e-10, "mixed": 2e-6}
# GMRES(m) in FP32: classical Gram-Schmidt loses orthogonality of the basis
# at a rate of u per step times the growth of the basis' condition number,
# and the least-squares correction inherits it; 5x the CG bar.
D_TOL_GMRES = {"fp64": 1e-10, "mixed": 1e-5}

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
        assert e <= D_TOL_GMRES[precision], (blk, e)
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


@pytest.mark.parametrize("name,precision,K,engine",
                         [("poisson256", "fp64", 50, "auto"), ("bumps512", "fp64", 8, "auto"),
                          ("bumps512", "mixed", 8, "auto"), ("bumps512", "fp64", 4, "phase"),
                          ("bumps512", "mixed", 4, "phase")])
def test_wholegrid_matched_sweeps(orc, name, precision, K, engine):
    """K synchronous sweeps from x = 0 in the benchmark's launch
    configuration against the oracle's K FP64 sweeps, on every cell, with
    the residual histories, on the default engine (the team engine here)
    and on the phase engine.  Mixed precision is held to the correction bar
    (the iterate is a sum of corrections, each refined by the next FP64
    residual)."""
    torch = torch_cuda()
    w = workload(name)
    shape, cuts = w["shape"], w["cuts"]
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    b = dev(w["b"])
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("wholegrid", name, precision, "K", K, engine)
    st = ms.ms_solve(h, b, x, 0.0, w["m"], "sync", max_sweeps=K, precision=precision,
                     history=K + 1, engine=engine)
    assert st.engine == ("team" if engine == "auto" else engine)
    xg = host(x)
    del x, b
    ms.ms_destroy(h)
    torch.cuda.empty_cache()
    assert st.status == 0 and st.sweeps == K
    beff = orc.lift_bc(w["b"], [None] * 6)
    _, xo, sw, _, hist = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=w["m"],
                                          max_sweeps=K)
    assert sw == K
    e = rel(xg, xo)
    bar = 1e-10 if precision == "fp64" else D_TOL["mixed"]
    assert e <= bar, e
    # histories: the residuals of iterates a relative delta apart differ by
    # at most ||A|| ||delta x|| / ||b_eff|| (||A|| <= 12)
    atol = 12 * max(e, 1e-13) * np.linalg.norm(xo) / np.linalg.norm(beff) + 1e-14
    np.testing.assert_allclose(st.history, hist, rtol=0, atol=atol)
    print(f"{name} {precision} K={K} {st.engine}: whole grid relative L2 {e:.2e}, final residual "
          f"{hist[-1]:.3e}")


def test_mixed_to_tolerance_matches_fp64_oracle_128(orc):
    """128^3 Poisson (f ~ N(0,1), seed 213), 4^3 blocks of 32^3, m = 10:
    the GPU's mixed-precision solve to 1e-8 against the oracle's FP64 solve
    to 1e-8, within 1e-6 relative L2; the oracle's FP64 residual of the GPU
    result meets the tolerance."""
    torch = torch_cuda()
    n = 128
    shape = (n, n, n)
    cuts = [inputs.uniform_cuts(n, 4)] * 3
    bh = inputs.poisson_randn(shape, 213)
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    say("mixed 128^3 to 1e-8")
    st = ms.ms_solve(h, dev(bh), x, 1e-8, 10, "sync", precision="mixed")
    xg = host(x)
    ms.ms_destroy(h)
    assert st.status == 0
    beff = orc.lift_bc(bh, [None] * 6)
    assert orc.residual(beff, xg) / np.linalg.norm(beff) <= 1e-8 * (1 + 1e-9)
    _, xo, sw, _, _ = orc.block_jacobi(beff, np.zeros(shape), cuts, tol=1e-8, m=10)
    e = rel(xg, xo)
    assert e <= 1e-6, e
    print(f"mixed 128^3: {st.sweeps} sweeps (oracle FP64 {sw}), vs FP64 oracle {e:.2e}")
