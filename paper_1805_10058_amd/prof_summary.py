"""Summaries of rocprofv3 output for the curl-div kernels.

    python -m paper_1805_10058_amd.prof_summary DIR [--top N] [--match SUBSTR]

DIR is a rocprofv3 output directory written with ``--output-format csv``.
Prints, per kernel, the dispatch count and average duration from
``*kernel_stats.csv`` and, when ``*counter_collection.csv`` files are present
(``--pmc`` runs), the average of every collected counter per dispatch.  With
``--by-grid`` the dispatches of ``*kernel_trace.csv`` and the counters are
split by grid size, which separates the levels of the multigrid hierarchy.
"""
import argparse
import collections
import csv
import glob
import os
import re
import sys


def _short(name):
    name = re.sub(r"\(anonymous namespace\)::", "", name)
    return re.sub(r"\((?:[^()]|\([^()]*\))*\)$", "", name).strip()


def kernel_stats(d):
    out = []
    for f in glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            out.append((_short(r["Name"]), int(r["Calls"]), float(r["AverageNs"]) / 1e3,
                        float(r["TotalDurationNs"]) / 1e6, float(r["Percentage"])))
    return sorted(out, key=lambda t: -t[3])


def by_grid(d):
    acc = collections.defaultdict(list)
    for f in glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            grid = r.get("Grid_Size", r.get("Grid_Size_X", "?"))
            dur = (float(r["End_Timestamp"]) - float(r["Start_Timestamp"])) / 1e3
            acc[(_short(r["Kernel_Name"]), grid)].append(dur)
    return sorted(((k[0], k[1], len(v), sum(v) / len(v), sum(v) / 1e3) for k, v in acc.items()),
                  key=lambda t: -t[4])


def counters(d, split_grid=False):
    acc = collections.defaultdict(lambda: collections.defaultdict(list))
    for f in glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True):
        for r in csv.DictReader(open(f)):
            name = _short(r.get("Kernel_Name", r.get("Kernel-Name", "?")))
            if split_grid:
                name = f"{name} grid {r.get('Grid_Size', '?')}"
            key = (name, r["Counter_Name"])
            acc[key][r.get("Dispatch_Id", r.get("Correlation_Id", ""))].append(float(r["Counter_Value"]))
    res = {}
    for key, per_dispatch in acc.items():
        vals = [sum(v) for v in per_dispatch.values()]  # sum over dimensions (XCDs, ...)
        res[key] = (len(vals), sum(vals) / len(vals))
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("dir")
    ap.add_argument("--top", type=int, default=25)
    ap.add_argument("--match", default="")
    ap.add_argument("--by-grid", action="store_true")
    a = ap.parse_args()
    if a.by_grid:
        rows = [r for r in by_grid(a.dir) if a.match in r[0]]
        print(f"{'kernel':80s} {'grid':>9s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>9s}")
        for name, grid, calls, avg, tot in rows[:a.top]:
            print(f"{name[:80]:80s} {grid:>9s} {calls:7d} {avg:9.2f} {tot:9.2f}")
        print()
    ks = [k for k in kernel_stats(a.dir) if a.match in k[0]]
    if ks:
        print(f"{'kernel':90s} {'calls':>7s} {'avg_us':>9s} {'total_ms':>9s} {'pct':>6s}")
        for name, calls, avg, tot, pct in ks[:a.top]:
            print(f"{name[:90]:90s} {calls:7d} {avg:9.2f} {tot:9.2f} {pct:6.2f}")
    cs = counters(a.dir, a.by_grid)
    if cs:
        print(f"{'kernel':90s} {'counter':>12s} {'dispatches':>10s} {'avg/dispatch':>14s}")
        for (name, cn), (nd, avg) in sorted(cs.items(), key=lambda kv: (-kv[1][1] * kv[1][0])):
            if a.match in name:
                print(f"{name[:90]:90s} {cn:>12s} {nd:10d} {avg:14.1f}")
    if not ks and not cs:
        print(f"no rocprofv3 csv output under {a.dir}", file=sys.stderr)
        sys.exit(1)


if __name__ == "__main__":
    main()
