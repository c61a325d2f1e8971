"""Benchmark: two-stage multisplitting sweeps on one MI355X.

Workload (default "bumps512"): 512^3 Poisson problem, source = 8 seeded
Gaussian bumps plus N(0, 1e-3) noise, zero Dirichlet boundaries, 8x8x8
blocks of 64^3, m = 10 inner CG iterations per block per sweep.  One "step"
is one outer sweep (residual with halo reads, 10 inner CG iterations on every
block, outer update), timed with tol <= 0 so exactly --steps sweeps run.
Inputs are resident in GPU memory before timing starts.

Prints one JSON line.  `value` is the algorithmic throughput of the
headline run (synchronous sweeps, mixed precision: FP32 inner CG, FP64
residual/test/update) in GB/s: the method's bytes per unknown per sweep (10
words per unknown per inner CG iteration plus the outer residual and update,
model_sweep_bytes) over the measured sweep time.  The library runs those
sweeps on its resident-team engine, which keeps a block's inner vectors on
chip; the phase-* modes run the same sweeps on the phase engine, whose
kernels stream every inner vector through memory (their compulsory bytes per
kernel: kernel_bytes).  The same line carries the FP64
and asynchronous sweeps, the global CG baseline, sweeps on overlapping blocks
(ovl-*, depth --ovl-depth), sweeps with GMRES inner solves (gmres-*), the
16-right-hand-side batched workload (batch-*), per-kernel event timings, the
dominant kernel's fraction of the 8 TB/s HBM peak beside two measured
ceilings (a device copy through HBM, and a copy of buffers that stay in the
256 MB on-package cache) with the HBM-streaming kernels listed apart, and
the CPU oracle timed on this host over a bounded sample of the same
workload (the only use of the oracle here).  After the timed region one
configuration (overlap 6, m = 30) is solved to the 1e-8 relative residual
with synchronous sweeps in mixed precision and in plain FP64, and with
asynchronous sweeps in mixed precision, and timed (time_to_tol; --tol-modes
picks them, --no-tol-solve skips them); the oracle then evaluates the FP64
residual of every final iterate on the host, as part of the CPU-baseline
leg.  With
--full-solve every mode is also run to 1e-8 and timed; the final residuals are
the library's own FP64 evaluation.

    python bench.py [--steps K] [--warmup W] [--modes sync-mixed,sync-fp64,...]
                    [--full-solve] [--no-cpu] [--no-tol-solve]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "time-to-1e-8 residual & stencil/CG HBM GB/s, 512^3 Laplace; mixed vs plain FP64"
# counter readings of the sweep kernels, reused only while the kernel
# sources are unchanged (paper_2009_12638_amd.pmc writes them)
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "hbm_traffic_bumps512.json")
HBM_PEAK_GBPS = 8000.0
# LDS bandwidth of the chip: 256 compute units x 128 bytes per clock x 2.4 GHz
LDS_PEAK_GBPS = 256 * 128 * 2.4
# Resident-team sweeps: HBM bytes per unknown a sweep must move (x and b
# read, x written; the inner vectors stay on chip) and LDS bytes per unknown
# per inner iteration (two stencil applies of p from LDS: 5 vector loads of VZ
# cells and 2 single-cell loads per VZ cells; p read and written once),
# VZ = 4 in FP32 and 2 in FP64.
TEAM_HBM_BYTES = 24


def team_lds_bytes(T: int) -> float:
    vz = 4 if T == 4 else 2
    return 2 * (5 + 2 / vz) * T + 2 * T
ALL_MODES = ["sync-mixed", "sync-fp64", "phase-mixed", "phase-fp64", "async-mixed",
             "async-fp64", "cg-fp64",
             "batch-mixed", "batch-fp64", "gmres-mixed", "gmres-fp64", "ovl-mixed", "ovl-fp64",
             "grad-fp64", "grad-mixed"]
DEFAULT_MODES = ("sync-mixed,sync-fp64,phase-mixed,phase-fp64,async-mixed,async-fp64,cg-fp64,"
                 "ovl-mixed,gmres-mixed,batch-mixed,grad-fp64")
BATCH_WORKLOAD = "uneven384"   # batched modes: 16 right-hand sides, uneven blocks
DIFF_WORKLOAD = "diff128"      # grad modes: forward + adjoint solve, 4^3 blocks of 32^3


def log(*a):
    print("[bench]", *a, file=sys.stderr, flush=True)


def kernel_bytes(m: int, T: int):
    """Compulsory bytes per unknown of each kernel launch in one synchronous
    sweep, in launch order, for inner type size T (8 = FP64, 4 = FP32):
    every operand vector counted once (halo re-reads are cache hits).

    resid   : read x, b (FP64), write r (T)
    stencil : read r (+ p_old after iteration 0), write p_new
    update  : read p, r (+ d after iteration 0), write d, r
    final   : read x_old, p (+ d after iteration 0), write x_new (FP64)
    """
    out = [("resid", 16 + T)]
    for j in range(m):
        out.append(("stencil", 2 * T if j == 0 else 3 * T))
        if j < m - 1:
            out.append(("update", 4 * T if j == 0 else 5 * T))
        else:
            out.append(("final", 16 + (T if j == 0 else 2 * T)))
    return out


def kernel_bytes_gmres(m: int, T: int):
    """Compulsory bytes per unknown of each launch of a synchronous sweep
    with GMRES(m) inner solves (per-block Hessenberg kernels move no vector):

    resid   : read x, b, write u_0
    stencil : Arnoldi step j, w = A v_j: read u_j, write w, read u_0..u_{j-1}
              for the dots (u_j counted once)
    orth    : read w and u_0..u_j, write u_{j+1}
    final   : read x_old and u_0..u_{m-1}, write x_new
    """
    out = [("resid", 16 + T)]
    for j in range(m):
        out.append(("stencil", (j + 2) * T))
        out.append(("orth", (j + 3) * T))
    out.append(("final", 16 + m * T))
    return out


def sweep_bytes(m: int, T: int, gmres: bool = False) -> int:
    return sum(b for _, b in (kernel_bytes_gmres if gmres else kernel_bytes)(m, T))


def model_sweep_bytes(m: int, mixed: bool) -> int:
    """Byte model of the method (10 words per unknown per CG iteration plus
    residual and update overhead), independent of this implementation."""
    return 40 * m + 40 if mixed else 80 * m + 48


CG_BYTES = {"stencil": 24, "update": 40}   # FP64 global CG, per unknown per iteration


def region_cells(shape, cuts, overlap: int) -> int:
    """Cells of the inner-solve boxes with overlap (each block grown across
    faces that have a neighbour, clipped to the grid); the grid size when
    overlap is 0."""
    # z grows by the overlap rounded up to the widest vector the z cuts allow
    vzb = next((w for w in (4, 2) if shape[2] % w == 0 and all(int(v) % w == 0 for v in cuts[2])),
               1)
    grow = [overlap, overlap, -(-overlap // vzb) * vzb]
    per_axis = []
    for n, c, gr in zip(shape, cuts, grow):
        c = [int(v) for v in c]
        per_axis.append([c[t + 1] - c[t] + min(gr, c[t]) + min(gr, n - c[t + 1])
                         for t in range(len(c) - 1)])
    total = 0
    for a in per_axis[0]:
        for b in per_axis[1]:
            for e in per_axis[2]:
                total += a * b * e
    return total


def per_kernel(prof, N, byte_lists, extra=None, cells=None):
    """Per kernel class: launches, average duration, compulsory GB/s and the
    unknowns one launch processes (launches cover groups of blocks).  cells:
    per class, the cells a pass touches (N unless overlap regions are on)."""
    out = {}
    for name, lst in byte_lists.items():
        N = (cells or {}).get(name, N)
        launches = prof.kernel_launches.get(name, 0)
        ms_tot = prof.kernel_ms.get(name, 0.0)
        if launches == 0 or ms_tot <= 0:
            continue
        bytes_tot = sum(lst) * N * prof.sweeps + (extra or {}).get(name, 0)
        passes = len(lst) * prof.sweeps + (1 if (extra or {}).get(name) else 0)
        out[name] = {"launches": launches, "avg_us": round(1e3 * ms_tot / launches, 2),
                     "total_ms": round(ms_tot, 3),
                     "GBps": round(bytes_tot / (ms_tot * 1e-3) / 1e9, 1),
                     "bytes_per_launch": int(bytes_tot / launches),
                     "unknowns_per_launch": int(round(N * passes / launches)),
                     "bytes_per_unknown": lst}
    return out


def grad_mode(args, torch, ms, mode: str):
    """One step = the differentiable solve of a least-squares loss: the
    forward solve to the workload's tol and, in backward, the adjoint solve
    (A is symmetric) to its adjoint tol, through torch.autograd."""
    from paper_2009_12638_amd import autograd, inputs
    precision = "mixed" if mode.endswith("mixed") else "fp64"
    T = 4 if precision == "mixed" else 8
    w = inputs.workload(DIFF_WORKLOAD)
    shape, cuts = w["shape"], w["cuts"]
    N = shape[0] * shape[1] * shape[2]
    m = args.grad_m or w["m"]
    ov = args.grad_overlap
    solver = autograd.PoissonSolver(shape, cuts=[list(map(int, c)) for c in cuts], tol=w["tol"],
                                    inner_iters=m, precision=precision,
                                    adjoint_tol=w["adjoint_tol"], overlap=ov)
    f = torch.tensor(w["f"], device="cuda", requires_grad=True)
    faces = [torch.tensor(g, device="cuda", requires_grad=True) for g in w["faces"]]
    ut = torch.tensor(w["ut"], device="cuda")

    def step():
        f.grad = None
        for g in faces:
            g.grad = None
        u = solver(f, faces)
        ((u - ut) ** 2).sum().backward()

    log(f"{mode}: warmup 1")
    step()
    K = max(1, min(args.steps, 3))
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(K):
        step()
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    fs, ad = solver.stats["forward"], solver.stats["adjoint"]
    log(f"{mode}: {K} forward + adjoint solves in {sec:.3f} s "
        f"({fs.sweeps} + {ad.sweeps} sweeps)")
    NR = region_cells(shape, cuts, ov)
    fin = dict(kernel_bytes(m, T))["final"]
    per_sweep = (sweep_bytes(m, T, False) - fin) * NR + fin * N
    return {"mode": mode, "workload": DIFF_WORKLOAD, "steps": K, "seconds": round(sec, 4),
            "ms_per_step": round(1e3 * sec / K, 3), "inner_iters": m, "overlap": ov,
            "forward_sweeps": fs.sweeps, "adjoint_sweeps": ad.sweeps,
            "forward_rel_residual": fs.rel_residual, "adjoint_rel_residual": ad.rel_residual,
            "tol": w["tol"], "adjoint_tol": w["adjoint_tol"],
            "GBps": round(per_sweep * (fs.sweeps + ad.sweeps) * K / sec / 1e9, 1)}


def run_mode(args, torch, ms, w, mode: str):
    kind, prec = mode.split("-")
    # phase-*: synchronous sweeps on the phase engine (the HBM-streaming
    # kernels); every other mode lets the library pick (the resident-team
    # engine wherever a block fits a team)
    engine = "auto"
    if kind == "phase":
        kind, engine = "sync", "phase"
    shape, cuts = w["shape"], w["cuts"]
    N = shape[0] * shape[1] * shape[2]
    m = args.m
    T = 4 if prec == "mixed" else 8
    precision = "mixed" if prec == "mixed" else "fp64"
    b = torch.from_numpy(w["b"]).to("cuda")
    nrhs = b.shape[0] if kind == "batch" else 1
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    # ovl-*: synchronous sweeps on overlapping blocks of depth --ovl-depth
    ov = (args.ovl_depth if kind == "ovl" else
          args.overlap if kind in ("sync", "async", "batch", "gmres") else 0)
    if ov:
        ms.ms_set_overlap(h, ov)
    if kind == "gmres":
        ms.ms_reserve_krylov(h, m)
    tuned = {}
    x = torch.zeros_like(b)
    if kind == "batch":
        ms.ms_reserve(h, nrhs)
    if kind in ("ovl", "batch") and args.autotune:
        from paper_2009_12638_amd import tune
        log(f"{mode}: autotuning overlap depth and m")
        torch.cuda.synchronize()
        t0 = time.perf_counter()

        def show(r):
            txt = f"{mode}: proxy o={r['overlap']} m={r['m']}: {r['sweeps']} sweeps, " \
                  f"{r['seconds']:.2f} s"
            if r["stopped"]:
                txt += " (stopped: slower than the best)"
            if "estimate" in r:
                txt += f"; full size {r['full_ms_per_sweep']:.1f} ms per sweep, " \
                       f"estimate {r['estimate']:.1f} s"
            log(txt)

        best, table = tune.tune_overlap_inner(shape, cuts, precision=precision, tol=w["tol"],
                                              progress=show, full=(h, b, x))
        ov, m = best["overlap"], best["m"]
        ms.ms_set_overlap(h, ov)
        x.zero_()
        tuned = {"overlap": ov, "inner_iters": m,
                 "tune_seconds": round(time.perf_counter() - t0, 2),
                 "table": [{k: (round(v, 4) if isinstance(v, float) else v) for k, v in r.items()}
                           for r in table]}
        log(f"{mode}: tuned overlap {ov}, m {m} in {tuned['tune_seconds']} s")
    NR = region_cells(shape, cuts, ov)   # cells the residual and inner kernels touch
    team_ok = False
    if kind == "ovl" and args.autotune:
        # the tile search concerns the phase engine (setting a tile option
        # selects it); skip it when the tuned pair runs on the team engine
        team_ok = ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=1,
                              precision=precision).engine == "team"
        x.zero_()
        if team_ok:
            log(f"{mode}: overlap {ov}, m {m} runs on the team engine: no tile search")
    if kind in ("ovl", "batch") and args.autotune and not team_ok:
        # tile shape with blocks per launch, on the real problem with the tuned m
        lay, lays = tune.tune_layout(
            h, b, x, precision, m=m, sweeps=2,
            progress=lambda r: log(f"{mode}: rows {r['rows']}, x chunk {r['x_chunk']}, "
                                   f"blocks per launch {r['group_blocks']}: "
                                   f"{r['ms_per_sweep']:.1f} ms per sweep"))
        log(f"{mode}: layout rows {lay['rows']}, x chunk {lay['x_chunk']}, blocks per launch "
            f"{lay['group_blocks']}: {lay['ms_per_sweep']:.1f} ms per sweep")
        tuned.update(rows=lay["rows"], x_chunk=lay["x_chunk"], group_blocks=lay["group_blocks"],
                     layout_table=[{k: (round(v, 2) if isinstance(v, float) else v)
                                    for k, v in r.items()} for r in lays])
    tile_kw = {k: tuned[k] for k in ("rows", "x_chunk", "group_blocks") if k in tuned}
    if args.inner_tol > 0 and kind in ("sync", "async", "ovl", "batch"):
        tile_kw["inner_tol"] = args.inner_tol

    def step(k, **kw):
        if kind == "cg":
            return ms.ms_cg(h, b, x, 0.0, k, **kw)
        if kind == "batch":
            return ms.ms_solve_batch(h, b, x, 0.0, m, max_sweeps=k, precision=precision,
                                     **tile_kw, **kw)[0]
        if kind == "gmres":
            return ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=k, precision=precision,
                               inner="gmres", **kw)
        return ms.ms_solve(h, b, x, 0.0, m, "sync" if kind == "ovl" else kind, max_sweeps=k,
                           precision=precision, engine=engine, **tile_kw, **kw)

    log(f"{mode}: warmup {args.warmup}")
    if args.warmup > 0:
        step(args.warmup)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = step(args.steps)
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    log(f"{mode}: {args.steps} steps in {sec:.3f} s")
    team = getattr(st, "engine", "") == "team"
    res = {"mode": mode, "steps": args.steps, "seconds": round(sec, 4),
           "ms_per_step": round(1e3 * sec / args.steps, 4), "nrhs": nrhs, "inner_iters": m,
           "engine": getattr(st, "engine", "") or "phase"}
    if args.inner_tol > 0:
        res["inner_tol"] = args.inner_tol   # GBps assume m iterations: an upper bound here
    if ov:
        res["overlap"] = ov
        res["region_cells"] = NR
    if tuned:
        res["autotuned"] = {k: tuned[k] for k in ("rows", "x_chunk", "group_blocks",
                                                  "inner_iters", "overlap", "tune_seconds",
                                                  "table", "layout_table") if k in tuned}
    if kind == "cg":
        bpu = sum(CG_BYTES.values())
        res["GBps"] = round(bpu * N * args.steps / sec / 1e9, 1)
        res["bytes_per_unknown_step"] = bpu
    elif team:
        # what the sweep moves through HBM (x, b over the inner-solve boxes,
        # x written)
        sweep_total = 16 * NR + 8 * N
        res["GBps"] = round(sweep_total * args.steps / sec / 1e9, 1)
        res["bytes_per_unknown_step"] = TEAM_HBM_BYTES
        res["model_GBps"] = round(model_sweep_bytes(m, T == 4) * N * args.steps / sec / 1e9, 1)
        res["unknown_iters_per_s"] = N * m * args.steps / sec
    else:
        gm = kind == "gmres"
        fin = dict((kernel_bytes_gmres if gm else kernel_bytes)(m, T))["final"]
        sweep_total = (sweep_bytes(m, T, gm) - fin) * NR + fin * N
        res["GBps"] = round(sweep_total * nrhs * args.steps / sec / 1e9, 1)
        res["bytes_per_unknown_step"] = sweep_bytes(m, T, gm)
        res["model_GBps"] = round(model_sweep_bytes(m, T == 4) * N * nrhs * args.steps / sec / 1e9, 1)
        res["unknown_iters_per_s"] = N * nrhs * m * args.steps / sec
    if kind == "async":
        res["max_staleness_seen"] = st.max_staleness_seen
        if st.block_sweeps:
            # sweeps each block did in the timed call (asynchronous blocks
            # need not end level)
            res["block_sweeps_min"] = int(min(st.block_sweeps))
            res["block_sweeps_max"] = int(max(st.block_sweeps))
    if team and kind in ("sync", "ovl"):
        # one cooperative launch per sweep: the method's bytes per unknown
        # per sweep, and the LDS bytes of the inner iterations
        prof = step(max(2, min(args.steps, 5)), profile=True)
        k = per_kernel(prof, N, {"other": [model_sweep_bytes(m, T == 4)]}).get("other")
        if k:
            k["bytes_per_unknown"] = [model_sweep_bytes(m, T == 4)]
            avg = k["avg_us"] * 1e-6
            k["hbm_GBps"] = round((16 * NR + 8 * N) / avg / 1e9, 1)
            k["hbm_bytes_per_launch"] = 16 * NR + 8 * N
            k["lds_bytes_per_launch"] = int(team_lds_bytes(T) * m * NR)
            k["lds_GBps"] = round(team_lds_bytes(T) * m * NR / avg / 1e9, 1)
            res["kernels"] = {"team": k}
    elif kind in ("sync", "cg", "batch", "gmres", "ovl"):
        prof = step(max(2, min(args.steps, 5)), profile=True)
        if kind in ("sync", "batch", "gmres", "ovl"):
            lists = {}
            for name, by in (kernel_bytes_gmres if kind == "gmres" else kernel_bytes)(m, T):
                lists.setdefault(name, []).append(by)
            cells = {"resid": NR * nrhs, "stencil": NR * nrhs, "update": NR * nrhs,
                     "orth": NR * nrhs, "final": N * nrhs}
            res["kernels"] = per_kernel(prof, N * nrhs, lists, extra={"resid": 16 * NR * nrhs},
                                        cells=cells)
        else:
            res["kernels"] = per_kernel(prof, N, {k: [v] for k, v in CG_BYTES.items()})
    if args.full_solve:
        x.zero_()
        log(f"{mode}: solve to {w['tol']}")
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        if kind == "cg":
            fs = ms.ms_cg(h, b, x, w["tol"], 100000)
            total = fs.sweeps
        elif kind == "batch":
            # in chunks with progress; right-hand sides that converged return
            # at once from the next chunk
            per = [0] * nrhs
            while True:
                sts = ms.ms_solve_batch(h, b, x, w["tol"], m, precision=precision,
                                        max_sweeps=args.chunk, raise_on_error=False, **tile_kw)
                for k, t in enumerate(sts):
                    per[k] += t.sweeps
                if all(t.status == ms.MS_OK for t in sts):
                    break
                if any(t.status not in (ms.MS_OK, ms.MS_ERR_NOT_CONVERGED) for t in sts) \
                        or max(per) > 200000:
                    raise RuntimeError(f"{mode}: batched solve failed")
                log(f"{mode}: {max(per)} sweeps, worst residual "
                    f"{max(t.rel_residual for t in sts):.3e}, {time.perf_counter() - t0:.1f} s")
            fs = sts[0]
            total = max(per)
            res["sweeps_to_tol_per_rhs"] = per
        else:
            # in chunks so progress is printed; a sweep resumed from x is the
            # same sweep (the whole outer state is x)
            total = inner_total = 0
            extra = {"inner": "gmres"} if kind == "gmres" else dict(tile_kw)
            while True:
                if kind != "gmres":
                    extra["engine"] = engine
                fs = ms.ms_solve(h, b, x, w["tol"], m,
                                 "sync" if kind in ("gmres", "ovl") else kind,
                                 precision=precision, max_sweeps=args.chunk,
                                 raise_on_error=False, **extra)
                total += fs.sweeps
                inner_total += fs.inner_iters
                if fs.status == ms.MS_OK:
                    break
                if fs.status != ms.MS_ERR_NOT_CONVERGED or total > 200000:
                    raise RuntimeError(f"{mode}: solve failed with status {fs.status}")
                log(f"{mode}: {total} sweeps, residual {fs.rel_residual:.3e}, "
                    f"{time.perf_counter() - t0:.1f} s")
        torch.cuda.synchronize()
        res["time_to_tol_s"] = round(time.perf_counter() - t0, 3)
        res["sweeps_to_tol"] = total
        if kind in ("sync", "async", "ovl") and total > 0:
            nb = (len(cuts[0]) - 1) * (len(cuts[1]) - 1) * (len(cuts[2]) - 1)
            res["mean_inner_iters"] = round(inner_total / (total * nb), 2)
        if kind == "batch":
            rels = [ms.ms_residual(h, b[k].contiguous(), x[k].contiguous())[0] for k in range(nrhs)]
            rel = max(rels)
        else:
            rel, _ = ms.ms_residual(h, b, x)
        res["final_rel_residual_gpu"] = rel
        log(f"{mode}: {total} sweeps, {res['time_to_tol_s']} s, residual {rel:.3e}")
    ms.ms_destroy(h)
    del x, b
    torch.cuda.empty_cache()
    return res


def overlap_study(args, torch, ms, inputs):
    """Sweeps and time to the workload's tolerance for several overlap depths
    (synchronous, mixed precision): the paper's overlap experiment on this
    GPU."""
    w = inputs.workload(args.study_workload)
    shape, cuts = w["shape"], w["cuts"]
    b = torch.from_numpy(w["b"]).to("cuda")
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    ms_list = [int(v) for v in args.study_m.split(",")] if args.study_m else [args.m]
    out = {"workload": args.study_workload, "tol": w["tol"], "precision": "mixed", "runs": []}
    for ov in [int(v) for v in args.overlap_study.split(",")]:
        ms.ms_set_overlap(h, ov)
        for m in ms_list:
            x = torch.zeros_like(b)
            ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=2, precision="mixed")  # warm
            x.zero_()
            torch.cuda.synchronize()
            t0 = time.perf_counter()
            total = 0
            while True:
                fs = ms.ms_solve(h, b, x, w["tol"], m, "sync", precision="mixed",
                                 max_sweeps=args.chunk, raise_on_error=False)
                total += fs.sweeps
                if fs.status == ms.MS_OK:
                    break
                if fs.status != ms.MS_ERR_NOT_CONVERGED or total > 200000:
                    raise RuntimeError(f"overlap {ov}, m {m}: solve failed, status {fs.status}")
            torch.cuda.synchronize()
            sec = time.perf_counter() - t0
            rel, _ = ms.ms_residual(h, b, x)
            out["runs"].append({"overlap": ov, "inner_iters": m, "sweeps_to_tol": total,
                                "seconds": round(sec, 3),
                                "ms_per_sweep": round(1e3 * sec / max(total, 1), 4),
                                "region_cells": region_cells(shape, cuts, ov),
                                "final_rel_residual": rel})
            log(f"overlap {ov}, m {m}: {total} sweeps, {sec:.2f} s, residual {rel:.3e}")
            del x
    ms.ms_destroy(h)
    del b
    torch.cuda.empty_cache()
    return out


def tol_solve(args, torch, ms, w, precision: str, mode: str = "sync"):
    """Time to the workload's tolerance for one configuration (overlap
    --tol-overlap, m = --tol-m, given precision and sweep mode; async with
    staleness 2), from x = 0.  Returns (record, final iterate on the host or
    None)."""
    shape, cuts = w["shape"], w["cuts"]
    b = torch.from_numpy(w["b"]).to("cuda")
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    if args.tol_overlap:
        ms.ms_set_overlap(h, args.tol_overlap)
    x = torch.zeros_like(b)
    ms.ms_solve(h, b, x, 0.0, args.tol_m, "sync", max_sweeps=2, precision=precision)
    x.zero_()
    log(f"time to {w['tol']}: overlap {args.tol_overlap}, m {args.tol_m}, {mode} {precision}")
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    total = 0
    while True:
        fs = ms.ms_solve(h, b, x, w["tol"], args.tol_m, mode, precision=precision,
                         max_sweeps=200, raise_on_error=False)
        total += fs.sweeps
        if fs.status == ms.MS_OK:
            break
        if fs.status != ms.MS_ERR_NOT_CONVERGED or total > 200000:
            raise RuntimeError(f"time-to-tol solve failed with status {fs.status}")
        log(f"  {total} sweeps, residual {fs.rel_residual:.3e}, {time.perf_counter() - t0:.1f} s")
    torch.cuda.synchronize()
    sec = time.perf_counter() - t0
    rel, _ = ms.ms_residual(h, b, x)
    out = {"mode": f"{mode}-{precision}", "engine": fs.engine or "phase",
           "overlap": args.tol_overlap,
           "inner_iters": args.tol_m, "tol": w["tol"], "sweeps": total,
           "seconds": round(sec, 3), "ms_per_sweep": round(1e3 * sec / max(total, 1), 3),
           "final_rel_residual_gpu": rel}
    if mode == "async":
        out["sweeps_note"] = "async: sweeps of the block that did most, summed over the calls"
        out["max_staleness_seen_last_call"] = fs.max_staleness_seen
    log(f"time to tol ({mode} {precision}): {total} sweeps, {sec:.2f} s, residual {rel:.3e}")
    xh = None if args.no_cpu else x.cpu().numpy()
    ms.ms_destroy(h)
    del x, b
    torch.cuda.empty_cache()
    return out, xh


def layout_study(args, torch, ms, inputs):
    """Sweeps and time to a tolerance for several block layouts of the study
    workload's grid (synchronous, mixed precision): the paper's comparison of
    2 blocks along x, 16 along x and 4x2x2 (Section 3.2) on this GPU."""
    w = inputs.workload(args.study_workload)
    shape = w["shape"]
    b = torch.from_numpy(w["b"]).to("cuda")
    out = {"workload": args.study_workload, "tol": args.layout_tol, "inner_iters": args.m,
           "precision": "mixed", "runs": []}
    for lay in args.layout_study.split(","):
        g = tuple(int(v) for v in lay.split("x"))
        h = ms.ms_create(shape, blocks=g)
        x = torch.zeros_like(b)
        ms.ms_solve(h, b, x, 0.0, args.m, "sync", max_sweeps=2, precision="mixed")  # warm
        x.zero_()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        st = ms.ms_solve(h, b, x, args.layout_tol, args.m, "sync", precision="mixed",
                         max_sweeps=200000)
        torch.cuda.synchronize()
        sec = time.perf_counter() - t0
        out["runs"].append({"blocks": lay, "sweeps_to_tol": st.sweeps, "seconds": round(sec, 3),
                            "ms_per_sweep": round(1e3 * sec / max(st.sweeps, 1), 4),
                            "final_rel_residual": st.rel_residual})
        log(f"layout {lay}: {st.sweeps} sweeps, {sec:.2f} s")
        ms.ms_destroy(h)
        del x
    del b
    torch.cuda.empty_cache()
    return out


def measured_traffic(kernel: str, unknowns_per_launch: int):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 counter
    summary (FETCH_SIZE and WRITE_SIZE, each scaled by what it reads for a
    plain copy of known size), or None when the kernels or the launch size
    changed since the counters were taken."""
    from paper_2009_12638_amd import pmc
    try:
        with open(TRAFFIC_FILE) as f:
            data = json.load(f)
        sha = pmc.source_sha1()
    except (OSError, ValueError):
        return None
    k = data.get("kernels", {}).get(kernel)
    if data.get("kernel_source_sha1") != sha or k is None:
        return None
    if k.get("unknowns_per_launch") != unknowns_per_launch:
        return None
    return k["fetch_bytes_per_launch"] + k["write_bytes_per_launch"]


def copy_peak(torch, gib: int = 1, reps: int = 5) -> float:
    """Measured device-to-device copy bandwidth (read + write bytes / time)
    over `reps` copies of `gib` GiB: the practical streaming ceiling beside
    the 8 TB/s data-sheet peak."""
    n = (gib << 30) // 8
    src = torch.ones(n, dtype=torch.float64, device="cuda")
    dst = torch.empty_like(src)
    dst.copy_(src)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        dst.copy_(src)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * 8 * n * reps / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del src, dst
    torch.cuda.empty_cache()
    return round(gbps, 1)


def cache_copy_peak(torch, mib: int = 48, reps: int = 60) -> float:
    """Measured copy bandwidth (read + write bytes / time) of a buffer pair
    that fits in the 256 MB on-package cache but not in the L2s (8 x 4 MB),
    copied back and forth `reps` times: the streaming ceiling of data that
    the inner iterations re-read from that cache."""
    n = (mib << 20) // 8
    a = torch.ones(n, dtype=torch.float64, device="cuda")
    c = torch.empty_like(a)
    for _ in range(4):
        c.copy_(a)
        a.copy_(c)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps // 2):
        c.copy_(a)
        a.copy_(c)
    e1.record()
    torch.cuda.synchronize()
    gbps = 2 * 8 * n * (reps // 2 * 2) / (e0.elapsed_time(e1) * 1e-3) / 1e9
    del a, c
    torch.cuda.empty_cache()
    return round(gbps, 1)


def team_roofline(head, ceilings):
    """Roofline of the resident-team sweep kernel (one launch per sweep).
    achieved: the method's bytes per unknown per sweep (10 words per unknown
    per CG iteration plus the outer residual and update) times the unknowns,
    over the launch's average duration; the kernel keeps the inner vectors on
    chip, so this exceeds what HBM could stream.  Beside it: the bytes the
    kernel does move through HBM (x and b read, x written) and the LDS bytes
    of its inner iterations against the chip's LDS bandwidth."""
    k = head["kernels"]["team"]
    prec = head["mode"].split("-")[1]
    tb = measured_traffic(f"team:{prec}", k["unknowns_per_launch"])
    avg = k["avg_us"] * 1e-6
    return {
        "bound": "hbm", "kernel": f"k_team ({head['mode']})",
        "achieved": k["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
        "frac": round(k["GBps"] / HBM_PEAK_GBPS, 4),
        "traffic": None if tb is None else round(tb / avg / 1e9, 1),
        "algorithmic_bytes_per_launch": k["bytes_per_launch"],
        "traffic_bytes_per_launch": None if tb is None else int(tb),
        "unknowns_per_launch": k["unknowns_per_launch"],
        "launch_avg_us": k["avg_us"],
        "note": ("achieved counts the method's streaming bytes (10 words per unknown per inner "
                 "iteration plus residual and update); the team kernel keeps r, d and p on chip "
                 "for all inner iterations, so frac above 1 is the factor by which it beats the "
                 "HBM roofline of the streaming formulation; traffic is what it does fetch and "
                 "write past the L2s"),
        "limited_by": ("the latency of the team sums (two per inner iteration, each a round trip "
                       "through the XCD's L2 for every team member) and LDS traffic; the x and b "
                       "reads run near the HBM share of a compute unit"),
        "hbm_moved": {"bytes_per_launch": k["hbm_bytes_per_launch"],
                      "bytes_per_unknown": TEAM_HBM_BYTES, "achieved": k["hbm_GBps"],
                      "frac": round(k["hbm_GBps"] / HBM_PEAK_GBPS, 4)},
        "lds": {"bytes_per_launch": k["lds_bytes_per_launch"], "achieved": k["lds_GBps"],
                "peak": round(LDS_PEAK_GBPS, 1),
                "frac": round(k["lds_GBps"] / LDS_PEAK_GBPS, 4)},
        "ceilings": ceilings,
    }


def phase_roofline(res, results, ceilings):
    """Roofline of the phase engine's dominant kernel (the HBM-streaming
    inner-iteration kernels), with the kernels that stream from HBM listed
    apart."""
    copy_gbps, cache_gbps = ceilings["hbm_copy_GBps"], ceilings["cache_resident_copy_GBps"]
    dom_name, dom = max(res["kernels"].items(), key=lambda kv: kv[1]["total_ms"])
    prec = res["mode"].split("-")[1]
    tb = (measured_traffic(f"{dom_name}:{prec}", dom["unknowns_per_launch"])
          if not res.get("overlap") and res.get("nrhs", 1) == 1 else None)
    roof = {"bound": "hbm", "kernel": f"k_{dom_name} ({res['mode']})",
            "achieved": dom["GBps"], "peak": HBM_PEAK_GBPS, "unit": "GB/s",
            "frac": round(dom["GBps"] / HBM_PEAK_GBPS, 4),
            "traffic": None if tb is None else round(tb / (dom["avg_us"] * 1e-6) / 1e9, 1),
            "algorithmic_bytes_per_launch": dom["bytes_per_launch"],
            "traffic_bytes_per_launch": None if tb is None else int(tb),
            "unknowns_per_launch": dom["unknowns_per_launch"],
            "launch_avg_us": dom["avg_us"],
            "served_from": ("the inner-iteration kernels (stencil, update) re-read their "
                            "launch group's vectors, sized to fit the 256 MB on-package "
                            "cache, so part of their traffic is served by that cache, not "
                            "HBM; traffic counts L2 misses (cache hits included); DRAM-side "
                            "bytes are not measured"),
            "ceilings": ceilings,
            "frac_of_cache_resident_copy": round(dom["GBps"] / cache_gbps, 4),
            "frac_of_hbm_copy": round(dom["GBps"] / copy_gbps, 4)}
    # the kernels that stream from HBM: outer residual, final update, global CG
    streaming = {}
    for mo, r in results.items():
        for kname in ("resid", "final") if mo == res["mode"] else ():
            k = r.get("kernels", {}).get(kname)
            if k:
                streaming[f"k_{kname} ({mo})"] = k["GBps"]
        if mo.startswith("cg-"):
            for kname, k in r.get("kernels", {}).items():
                streaming[f"k_gcg_{kname} ({mo})"] = k["GBps"]
    roof["hbm_streaming"] = {k: {"achieved": v, "frac_of_hbm_copy": round(v / copy_gbps, 4),
                                 "frac": round(v / HBM_PEAK_GBPS, 4)}
                             for k, v in streaming.items()}
    return roof


def cpu_model() -> str:
    try:
        with open("/proc/cpuinfo") as f:
            for ln in f:
                if ln.startswith("model name"):
                    return ln.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, m: int, sweeps: int, to_tol, finals, tol_overlap: int, tol_m: int,
                 ovl_sweeps: int):
    """The CPU oracle (test infrastructure, used here only as the reported
    baseline and as the independent check of the GPU's final iterates) on
    this host: `sweeps` FP64 sweeps of the workload with m inner iterations;
    `ovl_sweeps` FP64 sweeps of the time-to-tolerance configuration, whose
    per-sweep time times the GPU's FP64 sweep count is the oracle's
    extrapolated time to tolerance; and the oracle's FP64 relative residual
    of each final GPU iterate in `finals` (written into to_tol)."""
    import numpy as np
    import oracle
    o = oracle.load()
    beff = o.lift_bc(w["b"], [None] * 6)
    nb = float(np.linalg.norm(beff))
    shape, cuts = w["shape"], w["cuts"]
    N = shape[0] * shape[1] * shape[2]
    for prec, xh in finals.items():
        if xh is not None and prec in to_tol:
            to_tol[prec]["final_rel_residual_oracle"] = o.residual(beff, xh) / nb
            log(f"cpu oracle: residual of the GPU's {prec} iterate "
                f"{to_tol[prec]['final_rel_residual_oracle']:.4e}")
    log(f"cpu oracle: {sweeps} FP64 sweeps on {o.num_threads()} threads")
    t0 = time.perf_counter()
    o.block_jacobi(beff, np.zeros(shape), cuts, tol=0.0, m=m, max_sweeps=sweeps)
    sec = time.perf_counter() - t0
    out = {
        "value": round(model_sweep_bytes(m, False) * N * sweeps / sec / 1e9, 2),
        "unit": "GB/s",
        "cores": o.num_threads(),
        "kind": "oracle",
        "cpu_model": cpu_model(),
        "sample": f"{sweeps} FP64 synchronous sweeps of the full {shape[0]}^3 workload "
                  f"(m={m}): {sec:.2f} s, {1e3 * sec / sweeps:.0f} ms per sweep",
        "ms_per_sweep": round(1e3 * sec / sweeps, 1),
    }
    if ovl_sweeps > 0 and "fp64" in to_tol:
        log(f"cpu oracle: {ovl_sweeps} FP64 sweeps with overlap {tol_overlap}, m {tol_m}")
        t0 = time.perf_counter()
        o.multisplit(beff, np.zeros(shape), cuts, tol=0.0, m=tol_m, overlap=tol_overlap,
                     max_sweeps=ovl_sweeps)
        per = (time.perf_counter() - t0) / ovl_sweeps
        gs = to_tol["fp64"]["sweeps"]
        out["time_to_tol_extrapolated_s"] = round(per * gs, 1)
        out["time_to_tol_extrapolation"] = (
            f"extrapolated, not run: {ovl_sweeps} oracle FP64 sweeps with overlap {tol_overlap}, "
            f"m {tol_m} took {per:.2f} s each; times the {gs} sweeps the GPU's FP64 solve "
            f"needed to reach {to_tol['fp64']['tol']}")
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bumps512")
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--modes", default=DEFAULT_MODES)
    ap.add_argument("--full-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=16,
                    help="FP64 sweeps the CPU oracle baseline times (about 11 s at 512^3)")
    ap.add_argument("--chunk", type=int, default=400, help="sweeps per call in --full-solve")
    ap.add_argument("--autotune", action="store_true",
                    help="ovl and batched modes: pick the overlap depth and m first "
                         "(proxy solves with the same block shapes)")
    ap.add_argument("--inner-tol", type=float, default=0.0,
                    help="sync, async, ovl and batch modes: also stop a block's CG once its "
                         "residual fell by this factor (with --m as the cap)")
    ap.add_argument("--grad-m", type=int, default=0,
                    help="grad modes: inner iterations (0 = the workload's)")
    ap.add_argument("--grad-overlap", type=int, default=0, help="grad modes: overlap depth")
    ap.add_argument("--overlap", type=int, default=0,
                    help="overlap depth of the blocks in sync, async, batch and gmres modes")
    ap.add_argument("--ovl-depth", type=int, default=2,
                    help="overlap depth of the ovl-* modes")
    ap.add_argument("--overlap-study", default="",
                    help="comma list of overlap depths: solve the study workload to "
                         "tolerance for each (sync, mixed)")
    ap.add_argument("--study-workload", default="poisson256")
    ap.add_argument("--study-m", default="",
                    help="comma list of inner iteration counts for the overlap study "
                         "(default: --m)")
    ap.add_argument("--layout-study", default="",
                    help="comma list of block layouts GXxGYxGZ: solve the study workload to "
                         "--layout-tol for each (sync, mixed)")
    ap.add_argument("--layout-tol", type=float, default=1e-5)
    ap.add_argument("--no-tol-solve", action="store_true",
                    help="skip the time-to-tolerance solve of the default line")
    ap.add_argument("--tol-overlap", type=int, default=6)
    ap.add_argument("--tol-m", type=int, default=30)
    ap.add_argument("--tol-modes", default="sync-mixed,sync-fp64,async-mixed",
                    help="comma list of sweep mode and precision pairs solved to tolerance "
                         "(sync-mixed, sync-fp64, async-mixed, async-fp64)")
    ap.add_argument("--cpu-ovl-sweeps", type=int, default=2,
                    help="oracle sweeps of the time-to-tolerance configuration timed for its "
                         "extrapolated time to tolerance (0: skip)")
    ap.add_argument("--copy-probe", action="store_true",
                    help="also run a plain 1 GiB device copy (reference for hardware counters)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: the library has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)
    modes = [m for m in args.modes.split(",") if m]
    for m in modes:
        if m not in ALL_MODES:
            sys.exit(f"unknown mode {m}; choose from {ALL_MODES}")

    import torch
    from paper_2009_12638_amd import inputs, ms

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ms.lib()
    if args.copy_probe:
        src = torch.ones(1 << 27, dtype=torch.float64, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(2):
            dst.copy_(src)
        torch.cuda.synchronize()
        log("copy probe: 2 copies of 1 GiB")
        del src, dst
    log(f"building inputs for {args.workload}")
    w = inputs.workload(args.workload)
    results = {}
    wb = None
    for mo in modes:
        if mo.startswith("grad"):
            results[mo] = grad_mode(args, torch, ms, mo)
        elif mo.startswith("batch"):
            if wb is None:
                log(f"building inputs for {BATCH_WORKLOAD}")
                wb = inputs.workload(BATCH_WORKLOAD)
            results[mo] = run_mode(args, torch, ms, wb, mo)
        else:
            results[mo] = run_mode(args, torch, ms, w, mo)
    to_tol, finals = {}, {}
    if not args.no_tol_solve:
        for tm in [p for p in args.tol_modes.split(",") if p]:
            mode, prec = tm.split("-")
            key = prec if mode == "sync" else tm
            to_tol[key], finals[key] = tol_solve(args, torch, ms, w, prec, mode)
        if "mixed" in to_tol and "fp64" in to_tol:
            to_tol["fp64_over_mixed_time"] = round(to_tol["fp64"]["seconds"] /
                                                   to_tol["mixed"]["seconds"], 3)
    study = overlap_study(args, torch, ms, inputs) if args.overlap_study else None
    layouts = layout_study(args, torch, ms, inputs) if args.layout_study else None
    log("copy probe: device copy bandwidth (HBM) and cache-resident copy bandwidth")
    copy_gbps = copy_peak(torch)
    cache_gbps = cache_copy_peak(torch)
    head = results[modes[0]]
    roof = None
    ceilings = {"hbm_copy_GBps": copy_gbps, "cache_resident_copy_GBps": cache_gbps}
    hk = head.get("kernels") or {}
    if "team" in hk:
        roof = team_roofline(head, ceilings)
        ph = results.get("phase-" + head["mode"].split("-")[1])
        if ph and ph.get("kernels"):
            roof["streaming_engine"] = phase_roofline(ph, results, ceilings)
    elif hk:
        roof = phase_roofline(head, results, ceilings)
    cpu = None if args.no_cpu else cpu_baseline(w, args.m, args.cpu_sweeps, to_tol, finals,
                                                 args.tol_overlap, args.tol_m, args.cpu_ovl_sweeps)
    finals.clear()
    kind, prec = modes[0].split("-")
    if kind == "batch":
        w = wb
    shape = w["shape"]
    line = {
        "metric": METRIC,
        "value": head.get("model_GBps", head["GBps"]),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": head["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if prec == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": (f"{args.workload}: {shape[0]}x{shape[1]}x{shape[2]} Poisson, "
                         f"{len(w['cuts'][0]) - 1}^3 blocks of "
                         f"{shape[0] // (len(w['cuts'][0]) - 1)}^3, m={args.m}, "
                         f"{kind} sweeps, {prec}") if kind != "batch" else
                        (f"{BATCH_WORKLOAD}: {shape[0]}x{shape[1]}x{shape[2]} Poisson, "
                         f"{w['b'].shape[0]} right-hand sides, uneven blocks "
                         f"{[len(c) - 1 for c in w['cuts']]}, {prec}"),
            "step": "one outer sweep",
            "unknowns": shape[0] * shape[1] * shape[2],
            "engine": head.get("engine"),
            "value": ("the method's bytes per unknown per sweep (10 words per unknown per inner "
                      "CG iteration plus the outer residual and update: "
                      f"{model_sweep_bytes(args.m, prec == 'mixed')} B at m={args.m}) times the "
                      "unknowns, over the measured sweep time"),
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "modes": results,
    }
    if args.overlap:
        line["config"]["overlap"] = args.overlap
    if to_tol:
        line["time_to_tol"] = to_tol
    if study:
        line["overlap_study"] = study
    if layouts:
        line["layout_study"] = layouts
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
