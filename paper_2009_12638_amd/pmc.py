"""Summaries of rocprofv3 output for the measurement records.

    python -m paper_2009_12638_amd.pmc stats STATS_CSV TITLE COMMAND > kernels.md
    python -m paper_2009_12638_amd.pmc traffic FETCH_DIR WRITE_DIR BENCH_JSON OUT_JSON OUT_MD COMMAND

``stats`` turns a ``--kernel-trace --stats`` kernel_stats.csv into a table.

``traffic`` reads two ``--pmc`` runs of ``bench.py --copy-probe`` (one with
FETCH_SIZE, one with WRITE_SIZE; each counter is in KiB per dispatch) and the
JSON line that bench printed in one of them.  The counters are calibrated on
the 1 GiB device copies the bench makes (each reads and writes 1 GiB): the
scale factor of a counter is 1 GiB over its mean reading on those copies.
Every sweep kernel's scaled bytes per dispatch go to OUT_JSON, keyed by
kernel class and precision ("update:mixed", "team:fp64", ...) with the
unknowns one launch processes, and the hash of the kernel sources, so that
bench.py reuses them only while the kernels and launch sizes are unchanged.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = [os.path.join(HERE, "csrc", f)
                  for f in ("ms_kernels.hip", "ms_team.hip", "ms_device.h", "ms_tiles.h")]
COPY_KERNEL = "__amd_rocclr_copyBuffer"
COPY_BYTES = 1 << 30


def source_sha1() -> str:
    h = hashlib.sha1()
    for src in KERNEL_SOURCES:
        with open(src, "rb") as f:
            h.update(f.read())
    return h.hexdigest()


def short_name(name: str) -> str:
    """The kernel's name without its return type and parameter list."""
    name = name.split("(")[0].strip()
    return name[5:] if name.startswith("void ") else name


def kernel_class(name: str):
    """(class, precision) of a sweep kernel's demangled name, or None.
    k_update's fourth template argument marks the last inner step fused with
    the outer update; k_resid's marks the residual that writes r (the other
    instance only sums the residual for the convergence test)."""
    m = re.match(r"ms::k_(team|resid|stencil|update)<(float|double), ([^>]*)>", name)
    if not m:
        return None
    cls, t, rest = m.group(1), m.group(2), [a.strip() for a in m.group(3).split(",")]
    prec = "mixed" if t == "float" else "fp64"
    if cls == "update" and len(rest) >= 3 and rest[2] == "true":
        cls = "final"
    if cls == "resid" and len(rest) >= 3 and rest[2] != "true":
        return None
    return cls, prec


def read_counters(d: str, counter: str):
    """[(kernel name, value)] per dispatch from the counter csv under d."""
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = []
    for fn in files:
        with open(fn) as f:
            for r in csv.DictReader(f):
                if r.get("Counter_Name") == counter:
                    out.append((short_name(r["Kernel_Name"]), float(r["Counter_Value"])))
    return out


def scale(rows):
    """1 GiB over the mean reading of the 1 GiB copies (the copies reading
    at least half the largest copy's value)."""
    vals = [v for n, v in rows if n.startswith(COPY_KERNEL)]
    if not vals:
        raise RuntimeError("no device copies in the counter run (run bench with --copy-probe)")
    big = [v for v in vals if v >= 0.5 * max(vals)]
    return COPY_BYTES / (1024.0 * sum(big) / len(big)), len(big)


def launch_sizes(bench):
    """unknowns per launch of each (class, precision) from the bench line:
    team kernels from the sync-* modes, the others from phase-*."""
    out = {}
    for mode, res in bench.get("modes", {}).items():
        kind, prec = mode.split("-")
        for name, k in (res.get("kernels") or {}).items():
            if kind == "sync" and name == "team":
                out[("team", prec)] = k["unknowns_per_launch"]
            elif kind == "phase":
                out[(name, prec)] = k["unknowns_per_launch"]
    return out


def traffic(fetch_dir, write_dir, bench_json, out_json, out_md, command):
    fr, wr = read_counters(fetch_dir, "FETCH_SIZE"), read_counters(write_dir, "WRITE_SIZE")
    fs, nf = scale(fr)
    ws, nw = scale(wr)
    with open(bench_json) as f:
        line = [ln for ln in f if ln.startswith("{")][-1]
    bench = json.loads(line)
    sizes = launch_sizes(bench)
    agg = {}
    for rows, key in ((fr, "fetch"), (wr, "write")):
        for n, v in rows:
            a = agg.setdefault(n, {"fetch": [], "write": []})
            a[key].append(v)
    kernels = {}
    table = []
    for n, a in sorted(agg.items(), key=lambda kv: -len(kv[1]["fetch"])):
        fm = sum(a["fetch"]) / max(1, len(a["fetch"]))
        wm = sum(a["write"]) / max(1, len(a["write"]))
        kc = kernel_class(n)
        bpu = ""
        if kc and kc in sizes:
            fb, wb = fm * 1024 * fs, wm * 1024 * ws
            key = f"{kc[0]}:{kc[1]}"
            kernels[key] = {"fetch_bytes_per_launch": fb, "write_bytes_per_launch": wb,
                            "dispatches": len(a["fetch"]), "unknowns_per_launch": sizes[kc]}
            bpu = f"{(fb + wb) / sizes[kc]:.2f}"
        table.append(f"| `{n[:90]}` | {len(a['fetch'])} | {fm:.1f} | {wm:.1f} | {bpu} |")
    data = {"kernel_source_sha1": source_sha1(), "fetch_scale": fs, "write_scale": ws,
            "kernels": kernels}
    with open(out_json, "w") as f:
        json.dump(data, f, indent=1)
    md = [f"# HBM-side traffic per dispatch (rocprofv3 FETCH_SIZE / WRITE_SIZE), "
          f"{bench.get('config', {}).get('workload', '')}", "",
          "Commands (from /tmp, TMPDIR=/tmp, R = repository root), one counter per run:", "",
          f"    {command}", "",
          f"Calibration: the 1 GiB device copies ({nf} in the FETCH run, {nw} in the WRITE run) "
          f"read and write 1 GiB each; the scale factors are {fs:.4f} (fetch) and {ws:.4f} "
          f"(write).  FETCH_SIZE and WRITE_SIZE count traffic between the L2s and the fabric, "
          f"which includes hits in the on-package cache: DRAM-side bytes are not measured.", "",
          "| kernel | dispatches | FETCH KiB (raw mean) | WRITE KiB (raw mean) | "
          "scaled bytes/unknown |", "|---|---|---|---|---|"] + table
    with open(out_md, "w") as f:
        f.write("\n".join(md) + "\n")


def stats(csv_path, title, command):
    with open(csv_path) as f:
        rows = list(csv.DictReader(f))
    out = [f"# rocprofv3 kernel statistics: {title}", "",
           "Command (from /tmp, TMPDIR=/tmp, R = repository root):", "", f"    {command}", "",
           "| kernel | calls | total ms | avg us | min us | max us | % |",
           "|---|---|---|---|---|---|---|"]
    for r in rows:
        out.append(f"| `{short_name(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['MinNs']) / 1e3:.2f} | "
                   f"{float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f} |")
    print("\n".join(out))


if __name__ == "__main__":
    if len(sys.argv) >= 2 and sys.argv[1] == "stats" and len(sys.argv) == 5:
        stats(*sys.argv[2:])
    elif len(sys.argv) >= 2 and sys.argv[1] == "traffic" and len(sys.argv) == 8:
        traffic(*sys.argv[2:])
    else:
        sys.exit(__doc__)
