"""Summaries of rocprofv3 CSV output for this library's kernels.

    python -m paper_2005_07834_amd.profsum trace <kernel_trace.csv> [--match REGEX]
        per (kernel, grid size): dispatch count and mean / min / max duration in ms
    python -m paper_2005_07834_amd.profsum pmc <counter_collection.csv> [--match REGEX]
        per (kernel, grid size, counter): dispatch count and the mean value per dispatch
Groups of at most 8 dispatches (or --each N) also list every dispatch's own value, in dispatch
order; with --each N above 8, larger groups list their first N dispatches.

Launches of one kernel template on different column sets (site x grid, site x site) share a
name; the grid size (workgroups x threads) tells them apart, so both summaries group on it.
"""
from __future__ import annotations

import argparse
import collections
import csv
import re
import sys


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(f"none of {names} in the CSV header")


def _short(name: str) -> str:
    name = re.sub(r"\s+", " ", name)
    return name if len(name) <= 110 else name[:107] + "..."


def _grid(row) -> str:
    if "Grid_Size" in row:
        return row["Grid_Size"]
    return "x".join(row.get(f"Grid_Size_{a}", "1") for a in "XYZ")


def trace(path: str, match: str, each: int = 8) -> list[str]:
    groups = collections.defaultdict(list)
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = _col(r, "Kernel_Name")
            if not re.search(match, name):
                continue
            t = (int(_col(r, "End_Timestamp")) - int(_col(r, "Start_Timestamp"))) * 1e-6
            did = int(_col(r, "Dispatch_Id", "Correlation_Id"))
            groups[(_short(name), _grid(r))].append((did, t))
    out = [f"{'n':>4} {'mean_ms':>11} {'min_ms':>11} {'max_ms':>11}  grid  kernel"]
    for (name, grid), dts in sorted(groups.items(), key=lambda kv: -sum(t for _, t in kv[1])):
        ts = [t for _, t in sorted(dts)]
        out.append(f"{len(ts):4d} {sum(ts) / len(ts):11.3f} {min(ts):11.3f} {max(ts):11.3f}  "
                   f"{grid}  {name}")
        if len(ts) <= each:
            out.append("       each (ms): " + ", ".join(f"{t:.3f}" for t in ts))
        elif each > 8:
            out.append(f"       first {each} (ms): " + ", ".join(f"{t:.3f}" for t in ts[:each]))
    return out


def pmc(path: str, match: str, each: int = 8) -> list[str]:
    # (kernel, grid) -> counter -> dispatch -> value (summed over the rows of one dispatch)
    groups = collections.defaultdict(
        lambda: collections.defaultdict(lambda: collections.defaultdict(float)))
    with open(path, newline="") as fh:
        for r in csv.DictReader(fh):
            name = _col(r, "Kernel_Name")
            if not re.search(match, name):
                continue
            key = (_short(name), _grid(r))
            did = int(_col(r, "Dispatch_Id", "Correlation_Id"))
            groups[key][_col(r, "Counter_Name")][did] += float(_col(r, "Counter_Value"))
    out = [f"{'n':>4} {'counter':>28} {'mean_per_dispatch':>18}  grid  kernel"]
    for key, cs in groups.items():
        for cname, per in sorted(cs.items()):
            vals = [v for _, v in sorted(per.items())]
            out.append(f"{len(vals):4d} {cname:>28} {sum(vals) / len(vals):18.6e}  "
                       f"{key[1]}  {key[0]}")
            if len(vals) <= each:
                out.append("       each: " + ", ".join(f"{v:.6e}" for v in vals))
            elif each > 8:
                out.append(f"       first {each}: " + ", ".join(f"{v:.6e}" for v in vals[:each]))
    return out


def main(argv=None) -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("kind", choices=["trace", "pmc"])
    ap.add_argument("csv")
    ap.add_argument("--match", default=".")
    ap.add_argument("--each", type=int, default=8,
                    help="list every dispatch of groups up to this size, and the first this many "
                         "(in dispatch order) of larger groups when above 8")
    a = ap.parse_args(argv)
    lines = (trace if a.kind == "trace" else pmc)(a.csv, a.match, a.each)
    print("\n".join(lines))
    return 0


if __name__ == "__main__":
    sys.exit(main())
