"""Summaries of rocprofv3 output, for the files kept under profiles/.

    python -m paper_2512_04996_amd.profiling stats KERNEL_STATS_CSV OUT_MD --command "..."
        -> a short markdown table of per-kernel durations (average, calls, share)

    python -m paper_2512_04996_amd.profiling traffic --fetch DIR [DIR...] --write DIR [DIR...]
           --kernel NAME [NAME...] --copy-mib N --out OUT_JSON --command "..."
        -> HBM bytes per launch of each named kernel from FETCH_SIZE / WRITE_SIZE
           counter runs, each scaled by what the same counter reads for a plain
           copy of N MiB (the bytes a copy must move are known exactly); one
           entry per kernel under "variants" (several runs may be given, e.g.
           one per schedule, each ending with its own copy)

    python -m paper_2512_04996_amd.profiling counters DIR [DIR...] --kernels NAME... --out OUT_MD --command "..."
        -> per-kernel medians of every counter collected in the given runs

The counter runs must include one plain device-to-device copy of N MiB
(``bench.py --calib-copy-mib N``); its dispatch is the one whose kernel name
contains "copyBuffer".
"""
from __future__ import annotations

import argparse
import csv
import glob
import hashlib
import json
import os
import re
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))


def _short(name: str) -> str:
    m = re.search(r"(k_[A-Za-z0-9_]+(<[^>]*>)?)", name)
    if m:
        return m.group(1)
    return name.split("(")[0][:60]


def stats_table(csv_path: str, command: str, top: int = 20) -> str:
    rows = list(csv.DictReader(open(csv_path)))
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    lines = ["| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in rows[:top]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} | "
                     f"{float(r['MinNs']) / 1e3:.2f} | {float(r['MaxNs']) / 1e3:.2f} | {float(r['Percentage']):.2f}% |")
    return f"Command:\n\n```\n{command}\n```\n\n" + "\n".join(lines) + "\n"


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)
    if not files:
        raise FileNotFoundError(f"no counter_collection.csv under {d}")
    out = []
    for f in files:
        for r in csv.DictReader(open(f)):
            out.append(r)
    return out


def _per_dispatch(rows, counter: str):
    """{dispatch id: (kernel name, value)} summed over the counter's instances."""
    acc = {}
    for r in rows:
        cname = r.get("Counter_Name") or r.get("counter_name")
        if cname != counter:
            continue
        did = r.get("Dispatch_Id") or r.get("dispatch_id") or r.get("Correlation_Id")
        kname = r.get("Kernel_Name") or r.get("kernel_name") or ""
        val = float(r.get("Counter_Value") or r.get("counter_value") or 0.0)
        k, v = acc.get(did, (kname, 0.0))
        acc[did] = (kname, v + val)
    return acc


def traffic(fetch_dir: str, write_dir: str, kernel: str, copy_mib: float) -> dict:
    """One kernel's HBM bytes per launch from one FETCH_SIZE and one
    WRITE_SIZE run, or None when the runs hold no dispatch of it."""
    copy_bytes = copy_mib * 2 ** 20
    out = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        per = _per_dispatch(_counter_rows(d), counter)
        kv = [v for k, v in per.values() if kernel in k]
        cv = [v for k, v in per.values() if "copyBuffer" in k]
        if not kv:
            return None
        if not cv:
            raise RuntimeError(f"{counter}: no calibration copy in {d}")
        copy_reading = max(cv)                     # the large calibration copy
        scale = copy_bytes / (copy_reading * 1024.0)
        out[counter] = {"kernel_kib_per_dispatch": statistics.median(kv), "dispatches": len(kv),
                        "copy_kib": copy_reading, "scale": scale,
                        "bytes_per_launch": statistics.median(kv) * 1024.0 * scale}
    out["hbm_bytes_per_launch"] = out["FETCH_SIZE"]["bytes_per_launch"] + out["WRITE_SIZE"]["bytes_per_launch"]
    return out


def counters_table(dirs, kernels, command: str) -> str:
    """Median per dispatch of every counter found under the given counter
    directories, one column per kernel (matched by substring of its name)."""
    table = {}
    names = []
    for d in dirs:
        rows = _counter_rows(d)
        for cname in sorted({r.get("Counter_Name") or r.get("counter_name") for r in rows}):
            per = _per_dispatch(rows, cname)
            names.append(cname)
            for k in kernels:
                vals = [v for kn, v in per.values() if k in kn]
                table[(cname, k)] = (statistics.median(vals), len(vals)) if vals else None
    head = "| counter | " + " | ".join(f"`{k}`" for k in kernels) + " |"
    lines = [head, "|---|" + "---|" * len(kernels)]
    for cname in names:
        cells = []
        for k in kernels:
            v = table.get((cname, k))
            cells.append("-" if v is None else f"{v[0]:,.0f}")
        lines.append(f"| {cname} | " + " | ".join(cells) + " |")
    disp = []
    for k in kernels:
        ns = [table[(c, k)][1] for c in names if table.get((c, k))]
        disp.append(f"`{k}`: {max(ns) if ns else 0}")
    return (f"Command:\n\n```\n{command}\n```\n\nMedians over the dispatches of each kernel "
            f"({', '.join(disp)}), summed over the device.\n\n" + "\n".join(lines) + "\n")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("out")
    s.add_argument("--command", required=True)
    s.add_argument("--title", default="Kernel durations (rocprofv3 --kernel-trace --stats)")
    t = sub.add_parser("traffic")
    t.add_argument("--fetch", nargs="+", required=True)
    t.add_argument("--write", nargs="+", required=True)
    t.add_argument("--kernel", nargs="+", required=True)
    t.add_argument("--copy-mib", type=float, required=True)
    t.add_argument("--source", default=os.path.join(HERE, "csrc", "k_nns.hip"))
    t.add_argument("--out", required=True)
    t.add_argument("--command", required=True)
    c = sub.add_parser("counters")
    c.add_argument("dirs", nargs="+")
    c.add_argument("--kernels", nargs="+", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--command", required=True)
    c.add_argument("--title", default="Counters (rocprofv3 --pmc)")
    a = ap.parse_args(argv)
    if a.cmd == "counters":
        with open(a.out, "w") as f:
            f.write(f"# {a.title}\n\n" + counters_table(a.dirs, a.kernels, a.command))
        return 0
    if a.cmd == "stats":
        with open(a.out, "w") as f:
            f.write(f"# {a.title}\n\n" + stats_table(a.csv, a.command))
    else:
        if len(a.fetch) != len(a.write):
            raise SystemExit("give one --write run per --fetch run")
        variants = {}
        for fd, wd in zip(a.fetch, a.write):
            for k in a.kernel:
                r = traffic(fd, wd, k, a.copy_mib)
                if r is not None and k not in variants:
                    variants[k] = r
        missing = [k for k in a.kernel if k not in variants]
        if missing:
            raise SystemExit(f"no dispatch of {missing} in the given runs")
        res = {"variants": variants,
               "kernel_source_sha256": hashlib.sha256(open(a.source, "rb").read()).hexdigest(),
               "command": a.command}
        with open(a.out, "w") as f:
            json.dump(res, f, indent=1)
    return 0


if __name__ == "__main__":
    sys.exit(main())
