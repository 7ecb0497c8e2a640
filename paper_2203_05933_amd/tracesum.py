"""Summarise rocprofv3 CSV output of this library's kernels per launch shape.

rocprofv3's own --stats summary groups dispatches by kernel name only; one
kernel of this library runs with different grids (per tree level, per
workload), so this tool groups them by (kernel name, grid size) as well:

  python -m paper_2203_05933_amd.tracesum trace <run_kernel_trace.csv> [--match REGEX] [--last N]
      dispatches, average / median / min / max duration (microseconds)
  python -m paper_2203_05933_amd.tracesum pmc <run_counter_collection.csv> [--match REGEX] [--last N]
      median counter value per dispatch, per counter
  python -m paper_2203_05933_amd.tracesum traffic <fetch.csv> <write.csv> --calib REGEX --calib-mib M
                                                  [--match REGEX] [--last N]
      HBM bytes read and written per launch: the median FETCH_SIZE and
      WRITE_SIZE (KiB per dispatch, from two separate counter runs), each
      divided by what the same counter reads, per byte, for a calibration
      kernel (name matching --calib) that reads and writes M MiB

--last N keeps only the last N dispatches of every launch shape (in
dispatch order), e.g. the event-timed loop that ends a benchmark pass.

Prints a markdown table on stdout.  Reads text files only.
"""
from __future__ import annotations

import argparse
import csv
import re
import statistics
import sys
from collections import defaultdict


def _col(row, *names):
    for n in names:
        if n in row and row[n] != "":
            return row[n]
    raise KeyError(f"none of {names} in the CSV header")


def _short(name):
    # drop the argument list of a demangled kernel name, keep its template arguments
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            name = name[:i]
            break
    name = name.strip()
    if name.startswith("void "):
        name = name[5:]
    return name.replace("vp::", "")


def trace(path, match=None, last=None):
    groups = defaultdict(list)
    with open(path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(_col(r, "Dispatch_Id")))
    for row in rows:
        name = _short(_col(row, "Kernel_Name"))
        if match and not re.search(match, name):
            continue
        grid = int(_col(row, "Grid_Size_X", "Grid_Size"))
        dur = (int(_col(row, "End_Timestamp")) - int(_col(row, "Start_Timestamp"))) / 1e3
        groups[(name, grid)].append(dur)
    if last:
        groups = {k: v[-last:] for k, v in groups.items()}
    rows = sorted(groups.items(), key=lambda kv: -sum(kv[1]))
    print("| kernel | grid | dispatches | avg us | median us | min us | max us | total us |")
    print("|---|---|---|---|---|---|---|---|")
    for (name, grid), d in rows:
        print(f"| `{name}` | {grid} | {len(d)} | {statistics.fmean(d):.1f} | {statistics.median(d):.1f} | "
              f"{min(d):.1f} | {max(d):.1f} | {sum(d):.1f} |")


def pmc(path, match=None, last=None):
    groups = defaultdict(lambda: defaultdict(list))
    with open(path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(_col(r, "Dispatch_Id")))
    for row in rows:
        name = _short(_col(row, "Kernel_Name"))
        if match and not re.search(match, name):
            continue
        grid = int(_col(row, "Grid_Size", "Grid_Size_X"))
        groups[(name, grid)][_col(row, "Counter_Name")].append(float(_col(row, "Counter_Value")))
    if last:
        groups = {k: {c: v[-last:] for c, v in g.items()} for k, g in groups.items()}
    counters = sorted({c for g in groups.values() for c in g})
    print("| kernel | grid | dispatches | " + " | ".join(f"{c} (median)" for c in counters) + " |")
    print("|---|---|---|" + "---|" * len(counters))
    for (name, grid), g in sorted(groups.items(), key=lambda kv: kv[0]):
        n = max(len(v) for v in g.values())
        vals = " | ".join(f"{statistics.median(g[c]):.0f}" if c in g else "" for c in counters)
        print(f"| `{name}` | {grid} | {n} | {vals} |")


def _counter_medians(path, counter, last):
    groups = defaultdict(list)
    with open(path, newline="") as fh:
        rows = list(csv.DictReader(fh))
    rows.sort(key=lambda r: int(_col(r, "Dispatch_Id")))
    for row in rows:
        if _col(row, "Counter_Name") != counter:
            continue
        groups[(_short(_col(row, "Kernel_Name")), int(_col(row, "Grid_Size", "Grid_Size_X")))].append(
            float(_col(row, "Counter_Value")))
    if last:
        groups = {k: v[-last:] for k, v in groups.items()}
    return {k: (statistics.median(v), len(v)) for k, v in groups.items()}


def traffic(fetch_csv, write_csv, calib, calib_mib, match=None, last=None):
    fetch = _counter_medians(fetch_csv, "FETCH_SIZE", last)
    write = _counter_medians(write_csv, "WRITE_SIZE", last)
    kib = calib_mib * 1024.0

    def factor(table, what):
        hits = [v for (name, _), (v, _) in table.items() if re.search(calib, name)]
        if len(hits) != 1:
            raise SystemExit(f"{what}: {len(hits)} launch shapes match the calibration regex {calib!r}")
        return hits[0] / kib

    fr, fw = factor(fetch, "FETCH_SIZE"), factor(write, "WRITE_SIZE")
    print(f"calibration: FETCH_SIZE reads {fr:.4f} KiB per KiB read, WRITE_SIZE {fw:.4f} KiB per KiB written "
          f"({calib_mib} MiB each way)\n")
    print("| kernel | grid | dispatches | FETCH_SIZE KiB (median) | WRITE_SIZE KiB (median) | "
          "read MB (calibrated) | written MB (calibrated) |")
    print("|---|---|---|---|---|---|---|")
    keys = [k for k in fetch if k in write and not re.search(calib, k[0]) and (not match or re.search(match, k[0]))]
    keys.sort(key=lambda k: -(fetch[k][0] / fr + write[k][0] / fw))
    for k in keys:
        (f, n), (w, _) = fetch[k], write[k]
        print(f"| `{k[0]}` | {k[1]} | {n} | {f:.0f} | {w:.0f} | {f / fr * 1024 / 1e6:.1f} | "
              f"{w / fw * 1024 / 1e6:.1f} |")


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    ap.add_argument("kind", choices=["trace", "pmc", "traffic"])
    ap.add_argument("csv", nargs="+")
    ap.add_argument("--match", default=None, help="keep kernels whose short name matches this regex")
    ap.add_argument("--last", type=int, default=None, help="keep the last N dispatches of each launch shape")
    ap.add_argument("--calib", default=None, help="(traffic) regex naming the calibration kernel")
    ap.add_argument("--calib-mib", type=float, default=None, help="(traffic) MiB it reads and writes")
    a = ap.parse_args(argv)
    if a.kind == "traffic":
        if len(a.csv) != 2 or a.calib is None or a.calib_mib is None:
            ap.error("traffic takes <fetch.csv> <write.csv> --calib REGEX --calib-mib M")
        traffic(a.csv[0], a.csv[1], a.calib, a.calib_mib, a.match, a.last)
    elif len(a.csv) != 1:
        ap.error(f"{a.kind} takes one CSV")
    else:
        (trace if a.kind == "trace" else pmc)(a.csv[0], a.match, a.last)


if __name__ == "__main__":
    sys.exit(main())
