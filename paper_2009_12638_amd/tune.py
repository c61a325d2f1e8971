"""Autotuner for the multisplitting solve.

The paper fixes the number of inner iterations by hand and names run-time
auto-tuning of such parameters as future work (Sections 3.2 and 5).  This
module chooses, for one problem (grid, partition, precision, right-hand
sides):

* the tile shape (rows per thread, x chunk) together with the blocks per
  launch by timing a few sweeps of each pair,
* the overlap depth together with m by solving a smaller proxy problem
  with the same block shapes to tolerance for each pair, and
* the number of inner CG iterations m by the residual reduction each
  candidate achieves per second of solve time, measured from a common
  iterate past the initial transient.

It also runs solves whose inner-iteration count varies with the outer
iteration (Section 2.3 names a fixed or a varying count as a design choice):
an explicit schedule (solve_schedule), or one chosen while the solve runs
(solve_adaptive), which records the schedule it used.

Every timed run goes through the C ABI (ms_solve / ms_solve_batch); results
are cached in a JSON file keyed by the problem.
"""
from __future__ import annotations

import hashlib
import json
import math
import os
import time

import torch

from . import ms

DEFAULT_CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_2009_12638_amd",
                             "tune.json")
TILE_CANDIDATES = [(r, t) for r in (1, 2, 4) for t in (8, 16, 32)]
INNER_CANDIDATES = (5, 10, 20, 40)
OVERLAP_CANDIDATES = (0, 2, 4, 6, 8, 12)
OVERLAP_INNER_CANDIDATES = (10, 20, 30, 40, 60)
GROUP_CANDIDATES = (0, -1, 4, 16)


def problem_key(shape, cuts, precision, nrhs=1) -> str:
    dev = torch.cuda.get_device_name() if torch.cuda.is_available() else "cpu"
    raw = json.dumps([list(shape), [list(map(int, c)) for c in cuts], precision, nrhs, dev])
    return hashlib.sha1(raw.encode()).hexdigest()[:16]


def _run(h, b, x, sweeps, m, batch, **kw):
    if batch:
        return ms.ms_solve_batch(h, b, x, 0.0, m, max_sweeps=sweeps, **kw)
    return ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=sweeps, **kw)


def tune_layout(h, b, x, precision="mixed", m=10, sweeps=2, tiles=TILE_CANDIDATES,
                groups=GROUP_CANDIDATES, progress=None):
    """Fastest (rows, x_chunk, group_blocks) by wall time of `sweeps`
    synchronous sweeps, over every pair of tile shape and blocks per launch
    (the two interact: a grouping that is fast with one tile shape can be
    slow with another).  progress, if given, is called with each result."""
    batch = b.dim() == 4
    results = []
    for rows, tx in tiles:
        for g in groups:
            kw = dict(precision=precision, rows=rows, x_chunk=tx, group_blocks=g)
            _run(h, b, x, 1, m, batch, **kw)
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            _run(h, b, x, sweeps, m, batch, **kw)
            torch.cuda.synchronize()
            results.append(dict(rows=rows, x_chunk=tx, group_blocks=g,
                                ms_per_sweep=1e3 * (time.perf_counter() - t0) / sweeps))
            if progress:
                progress(results[-1])
    return min(results, key=lambda r: r["ms_per_sweep"]), results


def tune_inner(h, b, precision="mixed", candidates=INNER_CANDIDATES, warm_res=0.05,
               budget_s=0.5, tile=None, warm_max=300):
    """m with the largest log10 residual reduction per second, measured for
    each candidate from the same iterate (first one with residual <= warm_res
    under the default m), each for about budget_s seconds."""
    batch = b.dim() == 4
    tile = tile or {}
    kw = dict(precision=precision,
              **{k: tile[k] for k in ("rows", "x_chunk", "group_blocks") if k in tile})
    x0 = torch.zeros_like(b)
    if batch:
        ms.ms_solve_batch(h, b, x0, warm_res, 10, raise_on_error=False, max_sweeps=warm_max,
                          **kw)
    else:
        ms.ms_solve(h, b, x0, warm_res, 10, "sync", raise_on_error=False,
                    max_sweeps=warm_max, **kw)
    results = []
    for m in candidates:
        x = x0.clone()
        # sweeps that fit the budget, from one timed probe sweep
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        _run(h, b, x.clone(), 1, m, batch, **kw)
        torch.cuda.synchronize()
        per = max(time.perf_counter() - t0, 1e-5)
        sweeps = max(2, int(budget_s / per))
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        s = _run(h, b, x, sweeps, m, batch, history=sweeps + 1, **kw)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        hists = [t.history for t in s] if batch else [s.history]
        drop = min(math.log10(hh[0] / max(hh[-1], 1e-300)) for hh in hists)
        results.append(dict(m=m, sweeps=sweeps, seconds=sec, decades_per_s=drop / sec))
    best = max(results, key=lambda r: r["decades_per_s"])
    return best, results


def proxy_problem(shape, cuts, seed=7):
    """A smaller problem with the same block shapes: along each axis with more
    than two blocks, half of them (at least two), cut lists taken from the
    start of the original ones; a seeded N(0,1) source b = h^2 f."""
    pcuts = []
    for c in cuts:
        c = [int(v) for v in c]
        g = len(c) - 1
        keep = max(2, g // 2) if g > 2 else g
        pcuts.append(c[: keep + 1])
    pshape = tuple(c[-1] for c in pcuts)
    gen = torch.Generator().manual_seed(seed)
    h = 1.0 / (pshape[0] + 1)
    b = (h * h) * torch.randn(pshape, generator=gen, dtype=torch.float64)
    return pshape, pcuts, b


def tune_overlap_inner(shape, cuts, precision="mixed", overlaps=OVERLAP_CANDIDATES,
                       inners=OVERLAP_INNER_CANDIDATES, tol=1e-8, max_sweeps=20000,
                       progress=None, cutoff=1.5, chunk=100, full=None):
    """(overlap depth, m) pair that reaches tol fastest (the paper tunes the
    overlap and the inner iterations by hand, Section 3.2).

    The convergence curves of different pairs cross (few inner iterations
    win early, more win late), so short rate measurements mislead; instead
    every pair solves a proxy problem with the same block shapes
    (proxy_problem) to tol.  A pair still running after cutoff times the
    best time so far cannot win and is stopped (converged False, stopped
    True).

    full = (handle, b, x) of the real problem: the proxy then only supplies
    each pair's sweep count, and the cost of a sweep is timed on the real
    problem (two sweeps with that overlap and m; its overlap is left at the
    last candidate).  The proxy's blocks are mostly at the grid boundary,
    with fewer overlap slabs than interior blocks, so its own sweep times
    understate deep overlaps.  The pair with the smallest sweeps x real
    sweep time wins ("estimate" in the results).  Without full, the proxy's
    wall time decides.  progress, if given, is called with each pair's
    result as it completes.  Returns (best, results)."""
    pshape, pcuts, b_host = proxy_problem(shape, cuts)
    b = b_host.to("cuda")
    h = ms.ms_create(pshape, cuts=pcuts)
    results = []
    best_sec = None
    for ov in overlaps:
        ms.ms_set_overlap(h, ov)
        for m in inners:
            x = torch.zeros_like(b)
            ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=1, precision=precision)  # warm
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            total, stopped = 0, False
            while True:   # in chunks (a solve resumed from x is the same solve)
                s = ms.ms_solve(h, b, x, tol, m, "sync", max_sweeps=min(chunk, max_sweeps - total),
                                precision=precision, raise_on_error=False)
                total += s.sweeps
                if s.status != ms.MS_ERR_NOT_CONVERGED or total >= max_sweeps:
                    break
                if best_sec is not None and time.perf_counter() - t0 > cutoff * best_sec:
                    stopped = True
                    break
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            ok = s.status == ms.MS_OK
            r = dict(overlap=ov, m=m, sweeps=total, seconds=sec, converged=ok, stopped=stopped)
            if ok and (best_sec is None or sec < best_sec):
                best_sec = sec
            if full is not None and ok:
                fh, fb, fx = full
                ms.ms_set_overlap(fh, ov)
                batch = fb.dim() == 4
                _run(fh, fb, fx, 1, m, batch, precision=precision)
                torch.cuda.synchronize()
                t1 = time.perf_counter()
                _run(fh, fb, fx, 2, m, batch, precision=precision)
                torch.cuda.synchronize()
                r["full_ms_per_sweep"] = 1e3 * (time.perf_counter() - t1) / 2
                r["estimate"] = total * r["full_ms_per_sweep"] / 1e3
            results.append(r)
            if progress:
                progress(r)
    ms.ms_destroy(h)
    done = [r for r in results if r["converged"]] or results
    key = "estimate" if full is not None and all("estimate" in r for r in done) else "seconds"
    best = min(done, key=lambda r: r[key])
    return best, results


def autotune(shape, cuts, b, precision="mixed", cache=DEFAULT_CACHE, tune_m=True,
             refresh=False):
    """Tuned options {rows, x_chunk, group_blocks, inner_iters} for this
    problem, from the cache when present.  b: device tensor [nx,ny,nz] or
    [nrhs,nx,ny,nz]."""
    nrhs = b.shape[0] if b.dim() == 4 else 1
    key = problem_key(shape, cuts, precision, nrhs)
    db = {}
    if os.path.exists(cache):
        try:
            with open(cache) as f:
                db = json.load(f)
        except (OSError, ValueError):
            db = {}
    if key in db and not refresh:
        return db[key]
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts])
    if nrhs > 1:
        ms.ms_reserve(h, nrhs)
    x = torch.zeros_like(b)
    lay, lay_all = tune_layout(h, b, x, precision)
    out = dict(rows=lay["rows"], x_chunk=lay["x_chunk"], group_blocks=lay["group_blocks"],
               inner_iters=10, ms_per_sweep=lay["ms_per_sweep"], layouts=lay_all)
    if tune_m:
        inner, inner_all = tune_inner(h, b, precision, tile=lay)
        out["inner_iters"] = inner["m"]
        out["inner"] = inner_all
    ms.ms_destroy(h)
    db[key] = out
    os.makedirs(os.path.dirname(cache), exist_ok=True)
    tmp = cache + f".tmp{os.getpid()}"
    with open(tmp, "w") as f:
        json.dump(db, f, indent=1)
    os.replace(tmp, cache)
    return out


def solve_schedule(h, b, x, tol, schedule, mode="sync", **opts):
    """Synchronous solve whose inner-iteration count follows `schedule`, a
    list of (m, sweeps) pairs; the last m repeats until tol (or max_sweeps
    in total).  x is updated in place.  Returns (status, sweeps, residual)."""
    max_total = int(opts.pop("max_sweeps", 200000))
    total = 0
    st = None
    steps = list(schedule)
    while True:
        m, n = steps.pop(0) if len(steps) > 1 else (steps[0][0], max_total - total)
        n = min(n, max_total - total)
        st = ms.ms_solve(h, b, x, tol, m, mode, max_sweeps=n, raise_on_error=False, **opts)
        total += st.sweeps
        if st.status != ms.MS_ERR_NOT_CONVERGED or total >= max_total:
            return st.status, total, st.rel_residual


def solve_adaptive(h, b, x, tol, m0=10, m_min=2, m_max=64, chunk=200, max_sweeps=200000,
                   **opts):
    """Synchronous solve that picks the inner-iteration count while it runs.

    Sweeps run in chunks.  After each chunk the residual decay rate
    (decades per second, from the chunk's residual history and wall time)
    is compared with the previous chunk's: a step of m that made the rate
    better is repeated in the same direction, one that made it worse is
    undone and the direction reversed (m doubles or halves within
    [m_min, m_max]).  x is updated in place.

    Returns (status, total sweeps, final relative residual, schedule): the
    schedule lists the (m, sweeps) actually run, so the solve can be
    replayed exactly."""
    schedule = []
    total = 0
    m, prev_rate, direction = int(m0), None, 1
    while True:
        n = min(chunk, max_sweeps - total)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ms.ms_solve(h, b, x, tol, m, "sync", max_sweeps=n, history=n + 1,
                         raise_on_error=False, **opts)
        torch.cuda.synchronize()
        sec = max(time.perf_counter() - t0, 1e-9)
        schedule.append((m, st.sweeps))
        total += st.sweeps
        if st.status != ms.MS_ERR_NOT_CONVERGED or total >= max_sweeps:
            return st.status, total, st.rel_residual, schedule
        hist = st.history
        rate = math.log10(hist[0] / max(hist[-1], 1e-300)) / sec
        if prev_rate is not None and rate < prev_rate:
            direction = -direction          # that step hurt: go the other way
        prev_rate = rate
        m = max(m_min, min(m_max, m * 2 if direction > 0 else max(1, m // 2)))
