"""Summaries of rocprofv3 CSV output (kernel stats and HBM counters).

    python -m paper_2303_00123_amd.profsum stats <kernel_stats.csv> [--cmd "..."]
        Markdown table of per-kernel call counts and durations.

    python -m paper_2303_00123_amd.profsum counters --kernel k_tile <csv> [<csv> ...]
        Average per dispatch of every counter of a kernel over --pmc runs.

    python -m paper_2303_00123_amd.profsum traffic --kernel k_tile \\
        --fetch <dir>/..._counter_collection.csv --write <...csv> \\
        --copy-fetch <...csv> --copy-write <...csv> --copy-bytes B \\
        --algo-bytes A --out traffic.json [--cmd "..."]
        Per-dispatch HBM traffic of a kernel from FETCH_SIZE / WRITE_SIZE
        (KiB per dispatch), each scaled by the factor that maps the same
        counter onto the known byte count of a plain copy kernel.

The traffic record carries a hash of the kernel sources it was measured on
(`source_hash`), so a reader can tell when the kernel has changed since.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
TILE_SOURCES = ["csrc/qsv_tile.hip", "csrc/qsv_tile_core.h", "csrc/qsv_plan.cpp", "csrc/qsv_common.h",
                "csrc/qsv_internal.h", "csrc/qsv_jit.cpp"]


def source_hash(files=TILE_SOURCES) -> str:
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def kernel_stats(path: str):
    rows = []
    with open(path) as f:
        for r in csv.DictReader(f):
            rows.append(r)
    return rows


def stats_markdown(path: str, cmd: str = "", families=()) -> str:
    rows = kernel_stats(path)
    out = []
    if cmd:
        out.append(f"Command: `{cmd}`\n")
    if families:
        out.append("| kernel family (name prefix) | kernels | calls | total ms | avg us |")
        out.append("|---|---|---|---|---|")
        for fam in families:
            sel = [r for r in rows if r.get("Name", r.get("KernelName", "")).startswith(fam)]
            calls = sum(int(float(r.get("Calls", 0))) for r in sel)
            tot = sum(float(r.get("TotalDurationNs", 0)) for r in sel) / 1e6
            avg = tot * 1e3 / calls if calls else float("nan")
            out.append(f"| `{fam}` | {len(sel)} | {calls} | {tot:.3f} | {avg:.1f} |")
        out.append("")
    out.append("| kernel | calls | total ms | avg us | min us | max us | % |")
    out.append("|---|---|---|---|---|---|---|")
    for r in rows:
        name = r.get("Name", r.get("KernelName", "?"))
        calls = int(float(r.get("Calls", 0)))
        tot = float(r.get("TotalDurationNs", 0)) / 1e6
        avg = float(r.get("AverageNs", 0)) / 1e3
        mn = float(r.get("MinNs", 0)) / 1e3
        mx = float(r.get("MaxNs", 0)) / 1e3
        pct = float(r.get("Percentage", 0))
        out.append(f"| `{name[:90]}` | {calls} | {tot:.3f} | {avg:.1f} | {mn:.1f} | {mx:.1f} | {pct:.2f} |")
    return "\n".join(out) + "\n"


def counter_per_dispatch(path: str, kernel_substr: str, counter: str):
    vals = []
    with open(path) as f:
        for r in csv.DictReader(f):
            if kernel_substr in r["Kernel_Name"] and r["Counter_Name"] == counter:
                vals.append(float(r["Counter_Value"]))
    if not vals:
        raise ValueError(f"no {counter} rows for {kernel_substr} in {path}")
    return sum(vals) / len(vals), len(vals)


def counters_markdown(paths, kernel_substr: str, cmd: str = "") -> str:
    """Average per dispatch of every counter found for a kernel in one or
    more rocprofv3 counter_collection CSVs (one --pmc pass each)."""
    acc = {}
    for path in paths:
        with open(path) as f:
            for r in csv.DictReader(f):
                if kernel_substr in r["Kernel_Name"]:
                    acc.setdefault(r["Counter_Name"], []).append(float(r["Counter_Value"]))
    out = []
    if cmd:
        out.append(f"Command: `{cmd}`\n")
    out.append("| counter | dispatches | average per dispatch |")
    out.append("|---|---|---|")
    for k in sorted(acc):
        v = acc[k]
        out.append(f"| {k} | {len(v)} | {sum(v) / len(v):.6g} |")
    return "\n".join(out) + "\n"


def dispatches_markdown(path: str, cmd: str = "", prefix: str = "") -> str:
    """Per (kernel, grid size) duration statistics from a rocprofv3
    kernel_trace CSV: one kernel launched on different state sizes shows as
    one row per size."""
    groups = {}
    with open(path) as f:
        for r in csv.DictReader(f):
            name = r["Kernel_Name"]
            if prefix and prefix not in name:
                continue
            key = (name, int(r["Grid_Size_X"]))
            groups.setdefault(key, []).append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    out = []
    if cmd:
        out.append(f"Command: `{cmd}`\n")
    out.append("| kernel | grid (work-items) | calls | avg us | min us | max us |")
    out.append("|---|---|---|---|---|---|")
    for (name, grid), d in sorted(groups.items(), key=lambda kv: (-sum(kv[1]), kv[0])):
        out.append(f"| `{name[:90]}` | {grid} | {len(d)} | {sum(d) / len(d):.1f} | {min(d):.1f} | {max(d):.1f} |")
    return "\n".join(out) + "\n"


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd_", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--cmd", default="")
    s.add_argument("--family", action="append", default=[],
                   help="also total the kernels whose name starts with this prefix")
    c = sub.add_parser("counters")
    c.add_argument("--kernel", required=True)
    c.add_argument("--cmd", default="")
    c.add_argument("csv", nargs="+")
    d = sub.add_parser("dispatches")
    d.add_argument("csv")
    d.add_argument("--cmd", default="")
    d.add_argument("--kernel", default="", help="only kernels whose name contains this")
    t = sub.add_parser("traffic")
    t.add_argument("--kernel", required=True)
    t.add_argument("--fetch", required=True)
    t.add_argument("--write", required=True)
    t.add_argument("--copy-kernel", default="copy")
    t.add_argument("--copy-fetch", required=True)
    t.add_argument("--copy-write", required=True)
    t.add_argument("--copy-bytes", type=float, required=True)
    t.add_argument("--algo-bytes", type=float, required=True)
    t.add_argument("--out", required=True)
    t.add_argument("--cmd", default="")
    a = ap.parse_args(argv)
    if a.cmd_ == "stats":
        sys.stdout.write(stats_markdown(a.csv, a.cmd, a.family))
        return
    if a.cmd_ == "dispatches":
        sys.stdout.write(dispatches_markdown(a.csv, a.cmd, a.kernel))
        return
    if a.cmd_ == "counters":
        sys.stdout.write(counters_markdown(a.csv, a.kernel, a.cmd))
        return
    kf, nf = counter_per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")
    kw, nw = counter_per_dispatch(a.write, a.kernel, "WRITE_SIZE")
    cf, _ = counter_per_dispatch(a.copy_fetch, a.copy_kernel, "FETCH_SIZE")
    cw, _ = counter_per_dispatch(a.copy_write, a.copy_kernel, "WRITE_SIZE")
    # a copy of B bytes reads B and writes B
    f_scale = a.copy_bytes / (cf * 1024.0)
    w_scale = a.copy_bytes / (cw * 1024.0)
    fetch_b = kf * 1024.0 * f_scale
    write_b = kw * 1024.0 * w_scale
    rec = {
        "kernel": a.kernel,
        "fetch_kib_per_dispatch": kf, "write_kib_per_dispatch": kw, "dispatches": [nf, nw],
        "copy_fetch_kib": cf, "copy_write_kib": cw, "copy_bytes_each_way": a.copy_bytes,
        "fetch_scale": f_scale, "write_scale": w_scale,
        "traffic_bytes_per_launch": fetch_b + write_b,
        "algorithmic_bytes_per_launch": a.algo_bytes,
        "traffic_over_algorithmic": (fetch_b + write_b) / a.algo_bytes,
        "source_hash": source_hash(),
        "command": a.cmd,
    }
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
    print(json.dumps(rec))


if __name__ == "__main__":
    main()
