"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_2604_23175_amd.profiling stats  STATS_CSV  [--title T --command C]
    python -m paper_2604_23175_amd.profiling traffic FETCH_CSV WRITE_CSV --copy-mib M --out JSON

`stats` turns a `--kernel-trace --stats` kernel_stats.csv into a Markdown
table.  `traffic` reads two `--pmc FETCH_SIZE` / `--pmc WRITE_SIZE`
counter_collection.csv files (KiB per dispatch), calibrates them on the
plain device copy that `bench.py --copy-probe-mib M` performs first (its
dispatches must read and write exactly what they copy), and writes per-kernel
HBM bytes per launch together with a hash of the kernel source they were taken
on, which is what bench.py reports as `roofline.traffic`.
"""
from __future__ import annotations

import argparse
import collections
import csv
import hashlib
import json
import os
import re

HERE = os.path.dirname(os.path.abspath(__file__))
KERNELS = os.path.join(HERE, "csrc", "kernels.hip")


def kernels_sha() -> str:
    return hashlib.sha256(open(KERNELS, "rb").read()).hexdigest()[:16]


def short_name(name: str) -> str:
    """'void mase::k_eliminate<256>(mase::Dev, ...)' -> 'k_eliminate<256>'."""
    n = re.sub(r"\(.*$", "", name).replace("void ", "").strip()
    return n.split("::")[-1] if "mase::" in n else n


def per_dispatch(path: str, counter: str):
    """Counter value (summed over its dimensions) per dispatch, by kernel."""
    acc = collections.defaultdict(float)
    names = {}
    grids = {}
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] != counter:
            continue
        key = r["Dispatch_Id"]
        acc[key] += float(r["Counter_Value"])
        names[key] = short_name(r["Kernel_Name"])
        grids[key] = int(r["Grid_Size"])
    out = collections.defaultdict(list)
    for key, v in acc.items():
        out[names[key]].append((grids[key], v))
    return out


def traffic(fetch_csv: str, write_csv: str, copy_mib: int) -> dict:
    f = per_dispatch(fetch_csv, "FETCH_SIZE")
    w = per_dispatch(write_csv, "WRITE_SIZE")
    # the probe copy: the largest copy dispatches; each moves the same number
    # of bytes it reads and writes
    copies = sorted(v for _, v in f.get("__amd_rocclr_copyBuffer", []))
    wcopies = sorted(v for _, v in w.get("__amd_rocclr_copyBuffer", []))
    if not copies or not wcopies:
        raise SystemExit("no copy dispatches found: run bench.py with --copy-probe-mib")
    big_f = max(copies)
    big_w = max(wcopies)
    # the copy is split into equal dispatches; their size is a power-of-two
    # fraction of the probe
    kib = copy_mib * 1024.0
    while kib > big_f * 1.5:
        kib /= 2
    f_scale = kib / big_f
    w_scale = kib / big_w
    out = {"_calibration": {"copy_mib": copy_mib, "dispatch_kib": kib, "fetch_kib_measured": big_f,
                            "write_kib_measured": big_w, "fetch_scale": f_scale, "write_scale": w_scale}}
    sha = kernels_sha()
    for k in sorted(set(f) & set(w)):
        if not k.startswith("k_"):
            continue
        fv = [v for _, v in f[k]]
        wv = [v for _, v in w[k]]
        fk = sum(fv) / len(fv) * f_scale
        wk = sum(wv) / len(wv) * w_scale
        out[k] = {"fetch_kib": fk, "write_kib": wk, "bytes_per_launch": (fk + wk) * 1024.0,
                  "dispatches": len(fv), "kernels_sha": sha}
    return out


def stats_table(path: str, title: str = "", command: str = "") -> str:
    rows = list(csv.DictReader(open(path)))
    lines = []
    if title:
        lines.append(f"# {title}\n")
    if command:
        lines.append(f"Command: `{command}`\n")
    lines.append("| kernel | calls | total ms | average us | min us | max us | % |")
    lines.append("|---|---|---|---|---|---|---|")
    for r in rows:
        name = short_name(r["Name"])
        lines.append(f"| {name} | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.3f} | "
                     f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['MinNs']) / 1e3:.1f} | "
                     f"{float(r['MaxNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(lines) + "\n"


def last_dispatches(trace_csv: str, prefix: str, n: int) -> dict:
    """Mean / min / max duration (us) of the last n dispatches of the kernel
    whose short name starts with prefix, from a rocprofv3 kernel trace (the
    benchmark's per-stage profiled pass is the last work of its run)."""
    d = []
    for r in csv.DictReader(open(trace_csv)):
        if short_name(r["Kernel_Name"]).startswith(prefix):
            d.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    d.sort()
    w = [x[1] / 1e3 for x in d[-n:]]
    return {"kernel_prefix": prefix, "dispatches": len(w), "mean_us": sum(w) / max(1, len(w)),
            "min_us": min(w) if w else 0.0, "max_us": max(w) if w else 0.0}


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    s = sub.add_parser("stats")
    s.add_argument("csv")
    s.add_argument("--title", default="")
    s.add_argument("--command", default="")
    t = sub.add_parser("traffic")
    t.add_argument("fetch_csv")
    t.add_argument("write_csv")
    t.add_argument("--copy-mib", type=int, required=True)
    t.add_argument("--out", required=True)
    ls = sub.add_parser("last")
    ls.add_argument("trace_csv")
    ls.add_argument("prefix")
    ls.add_argument("n", type=int)
    a = ap.parse_args()
    if a.cmd == "last":
        print(json.dumps(last_dispatches(a.trace_csv, a.prefix, a.n)))
    elif a.cmd == "stats":
        print(stats_table(a.csv, a.title, a.command), end="")
    else:
        res = traffic(a.fetch_csv, a.write_csv, a.copy_mib)
        with open(a.out, "w") as fh:
            json.dump(res, fh, indent=1)
        print(json.dumps(res, indent=1))


if __name__ == "__main__":
    main()
