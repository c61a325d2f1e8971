"""Benchmark: synchronous two-stage multisplitting sweeps on one MI355X.

Workload (default "bumps512"): 512^3 Poisson problem, source = 8 seeded
Gaussian bumps plus N(0, 1e-3) noise, zero Dirichlet boundaries, 8x8x8
blocks of 64^3, m = 10 inner CG iterations per block per sweep.  One "step"
is one outer sweep (residual with halo reads, 10 inner CG iterations on every
block, outer update), timed with tol <= 0 so exactly --steps sweeps run.
Inputs are resident in GPU memory before timing starts.

Prints one JSON line.  `value` is the whole-sweep memory throughput of the
headline precision (mixed: FP32 inner CG, FP64 outer) in GB/s, using the
compulsory bytes per unknown of the kernels that make up a sweep (see
sweep_bytes); the FP64 sweep is reported beside it, with per-kernel event
timings, the dominant kernel's fraction of the 8 TB/s HBM peak, and the CPU
oracle timed on this host over a bounded sample of the same workload.

    python bench.py [--steps K] [--warmup W] [--precision mixed|fp64|both]
                    [--full-solve] [--no-cpu]
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
HBM_PEAK_GBPS = 8000.0


def kernel_bytes(m: int, T: int):
    """Compulsory bytes per unknown of each kernel launch in one sweep, in
    launch order, for inner type size T (8 = FP64, 4 = FP32): every operand
    vector counted once (halo re-reads are cache hits and not counted).

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


def sweep_bytes(m: int, T: int) -> int:
    return sum(b for _, b in kernel_bytes(m, T))


def model_sweep_bytes(m: int, mixed: bool) -> int:
    """Byte model of the method (10 words per unknown per CG iteration plus
    residual and update overhead), independent of this implementation."""
    return 40 * m + 40 if mixed else 80 * m + 48


def run_gpu(args, torch, ms, inputs, w, precision: str):
    shape, cuts = w["shape"], w["cuts"]
    N = shape[0] * shape[1] * shape[2]
    m = args.m
    T = 4 if precision == "mixed" else 8
    b = torch.from_numpy(w["b"]).to("cuda")
    h = ms.ms_create(shape, cuts=[list(map(int, c)) for c in cuts], faces=None)
    x = torch.zeros(shape, dtype=torch.float64, device="cuda")
    print(f"[bench] {precision}: warmup {args.warmup} sweeps", file=sys.stderr, flush=True)
    if args.warmup > 0:
        ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=args.warmup, precision=precision)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    st = ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=args.steps, precision=precision)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    sec = t1 - t0
    print(f"[bench] {precision}: {args.steps} sweeps in {sec:.3f} s", file=sys.stderr, flush=True)
    # per-kernel event timing in a separate, shorter run (events perturb a little)
    prof = ms.ms_solve(h, b, x, 0.0, m, "sync", max_sweeps=max(2, min(args.steps, 5)),
                       precision=precision, profile=True)
    kb = kernel_bytes(m, T)
    per_class_bytes = {}
    for name, by in kb:
        per_class_bytes.setdefault(name, []).append(by)
    kernels = {}
    for name, lst in per_class_bytes.items():
        launches = prof.kernel_launches.get(name, 0)
        ms_tot = prof.kernel_ms.get(name, 0.0)
        if launches == 0 or ms_tot <= 0:
            continue
        # bytes of all launches of this class in the profiled run: each sweep
        # runs the class's per-cell byte list over every unknown
        sweeps_prof = prof.sweeps
        bytes_tot = sum(lst) * N * sweeps_prof
        if name == "resid":
            bytes_tot += 16 * N      # residual-only check of the final iterate
        kernels[name] = {
            "launches": launches,
            "avg_us": 1e3 * ms_tot / launches,
            "total_ms": ms_tot,
            "GBps": bytes_tot / (ms_tot * 1e-3) / 1e9,
            "bytes_per_unknown": lst,
        }
    res = {
        "precision": precision,
        "sweeps": st.sweeps,
        "seconds": sec,
        "ms_per_sweep": 1e3 * sec / args.steps,
        "GBps": sweep_bytes(m, T) * N * args.steps / sec / 1e9,
        "bytes_per_unknown_sweep": sweep_bytes(m, T),
        "model_GBps": model_sweep_bytes(m, precision == "mixed") * N * args.steps / sec / 1e9,
        "unknown_iters_per_s": N * m * args.steps / sec,
        "kernels": kernels,
    }
    if args.full_solve:
        x.zero_()
        print(f"[bench] {precision}: full solve to {w['tol']}", file=sys.stderr, flush=True)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        fs = ms.ms_solve(h, b, x, w["tol"], m, "sync", precision=precision)
        torch.cuda.synchronize()
        t1 = time.perf_counter()
        rel, _ = ms.ms_residual(h, b, x)
        res["time_to_tol_s"] = t1 - t0
        res["sweeps_to_tol"] = fs.sweeps
        res["final_rel_residual"] = rel
    ms.ms_destroy(h)
    del x, b
    torch.cuda.empty_cache()
    return res


def cpu_baseline(w, m: int, sweeps: int):
    import numpy as np

    import oracle
    o = oracle.load()
    shape, cuts = w["shape"], w["cuts"]
    N = shape[0] * shape[1] * shape[2]
    beff = o.lift_bc(w["b"], [None] * 6)
    x0 = np.zeros(shape)
    print(f"[bench] cpu oracle: {sweeps} FP64 sweeps on {o.num_threads()} threads",
          file=sys.stderr, flush=True)
    t0 = time.perf_counter()
    st, x, sw, inner, hist = o.block_jacobi(beff, x0, cuts, tol=0.0, m=m, max_sweeps=sweeps)
    sec = time.perf_counter() - t0
    return {
        "value": sweep_bytes(m, 8) * N * sweeps / sec / 1e9,
        "unit": "GB/s",
        "cores": o.num_threads(),
        "kind": "oracle",
        "sample": f"{sweeps} FP64 sweeps of the full {shape[0]}^3 workload (m={m}), "
                  f"{sec:.2f} s, {1e3 * sec / sweeps:.0f} ms per sweep",
        "ms_per_sweep": 1e3 * sec / sweeps,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="bumps512")
    ap.add_argument("--m", type=int, default=10)
    ap.add_argument("--precision", default="both", choices=["both", "mixed", "fp64"])
    ap.add_argument("--full-solve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--cpu-sweeps", type=int, default=4)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              f"(asked for --gpus {args.gpus})", file=sys.stderr)
        sys.exit(2)

    import torch
    from paper_2009_12638_amd import inputs, ms

    if not torch.cuda.is_available():
        print("bench.py needs a GPU", file=sys.stderr)
        sys.exit(1)
    ms.lib()
    print(f"[bench] building inputs for {args.workload}", file=sys.stderr, flush=True)
    w = inputs.workload(args.workload)
    precs = ["mixed", "fp64"] if args.precision == "both" else [args.precision]
    results = {p: run_gpu(args, torch, ms, inputs, w, p) for p in precs}
    head = results[precs[0]]
    # roofline of the dominant kernel (largest total time) of the headline run
    dom_name, dom = max(head["kernels"].items(), key=lambda kv: kv[1]["total_ms"])
    roof = {
        "bound": "hbm",
        "kernel": f"k_{dom_name} ({head['precision']})",
        "achieved": round(dom["GBps"], 1),
        "peak": HBM_PEAK_GBPS,
        "unit": "GB/s",
        "frac": round(dom["GBps"] / HBM_PEAK_GBPS, 4),
        "traffic": None,
    }
    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, args.m, args.cpu_sweeps)
    shape = w["shape"]
    line = {
        "metric": METRIC,
        "value": round(head["GBps"], 1),
        "unit": "GB/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_sweep"], 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32+f64" if head["precision"] == "mixed" else "f64",
        "data": "synthetic",
        "config": {
            "workload": f"{args.workload}: {shape[0]}x{shape[1]}x{shape[2]} Poisson, "
                        f"{len(w['cuts'][0]) - 1}^3 blocks, m={args.m}, sync sweeps",
            "step": "one outer sweep",
            "unknowns": shape[0] * shape[1] * shape[2],
        },
        "roofline": roof,
        "cpu_baseline": cpu,
        "modes": results,
    }
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
