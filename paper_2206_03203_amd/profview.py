"""Per-kernel tables from rocprofv3 CSV output, for reading the library's
profiles.

    python -m paper_2206_03203_amd.profview trace KERNEL_TRACE.csv [--top N]
    python -m paper_2206_03203_amd.profview counters --trace KERNEL_TRACE.csv \\
        COUNTER_COLLECTION.csv [...] [--fetch-scale F] [--write-scale W] [--top N]

Rows are keyed by kernel (template arguments kept, argument list dropped)
and grid size, so the same kernel on different levels or systems stays
apart.  ``trace`` lists launches and mean duration per key.  ``counters``
joins any number of counter runs (one counter group per run) to a trace of
the same command: the mean of every counter per launch and, when FETCH_SIZE
and WRITE_SIZE (KiB per dispatch) are present, the HBM bytes per launch
scaled by the factors measured on a plain copy kernel, the rate those bytes
give over the traced duration, and the L2 hit fraction from TCC_HIT_sum and
TCC_MISS_sum.  Dispatches before the last ``cache_flush_kernel`` (the
autotuner's cold-cache reads at set-up) are left out."""

from __future__ import annotations

import argparse
import collections
import csv
import re
import sys


def kernel_key(name: str) -> str:
    name = name.replace("void ", "").replace("mdp::(anonymous namespace)::", "").replace("mdp::", "")
    depth = 0
    for i, ch in enumerate(name):
        if ch == "<":
            depth += 1
        elif ch == ">":
            depth -= 1
        elif ch == "(" and depth == 0:
            return name[:i].strip()
    return name.strip()


def _grid(row) -> int:
    for k in ("Grid_Size", "Grid_Size_X"):
        if k in row and row[k] != "":
            return int(row[k])
    return 0


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def _after_flush(rows, order_key):
    last = max([int(r[order_key]) for r in rows if "cache_flush" in r["Kernel_Name"]] or [-1])
    return [r for r in rows if int(r[order_key]) > last]


def trace_table(path):
    rows = _after_flush(_rows(path), "Start_Timestamp")
    agg = collections.defaultdict(lambda: [0, 0.0])
    for r in rows:
        k = (kernel_key(r["Kernel_Name"]), _grid(r))
        agg[k][0] += 1
        agg[k][1] += (int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3
    return agg  # (kernel, grid) -> [launches, total us]


def counter_table(paths):
    agg = collections.defaultdict(lambda: collections.defaultdict(list))
    for p in paths:
        rows = _rows(p)
        key = "Dispatch_Id" if rows and "Dispatch_Id" in rows[0] else "Correlation_Id"
        for r in _after_flush(rows, key):
            agg[(kernel_key(r["Kernel_Name"]), _grid(r))][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return agg  # (kernel, grid) -> counter -> values per dispatch


def main(argv=None) -> int:
    ap = argparse.ArgumentParser(description=__doc__, formatter_class=argparse.RawDescriptionHelpFormatter)
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("csv")
    t.add_argument("--top", type=int, default=60)
    c = sub.add_parser("counters")
    c.add_argument("--trace", required=True)
    c.add_argument("csv", nargs="+")
    c.add_argument("--fetch-scale", type=float, default=2.0)
    c.add_argument("--write-scale", type=float, default=1.0)
    c.add_argument("--top", type=int, default=40)
    c.add_argument("--match", default="", help="regular expression the kernel name must match")
    a = ap.parse_args(argv)
    tr = trace_table(a.trace if a.cmd == "counters" else a.csv)
    total = sum(v[1] for v in tr.values())
    order = sorted(tr.items(), key=lambda kv: -kv[1][1])
    if a.cmd == "trace":
        print(f"kernel time after set-up: {total / 1e3:.2f} ms over {sum(v[0] for v in tr.values())} dispatches")
        print(f"{'total_ms':>9} {'launches':>8} {'avg_us':>8} {'grid':>9}  kernel")
        for (k, g), (n, us) in order[: a.top]:
            print(f"{us / 1e3:9.2f} {n:8d} {us / n:8.2f} {g:9d}  {k}")
        return 0
    ct = counter_table(a.csv)
    names = sorted({c for v in ct.values() for c in v})
    extra = [c for c in names if c not in ("FETCH_SIZE", "WRITE_SIZE", "TCC_HIT_sum", "TCC_MISS_sum")]
    print(f"kernel time after set-up: {total / 1e3:.2f} ms; HBM bytes = FETCH_SIZE x {a.fetch_scale} + "
          f"WRITE_SIZE x {a.write_scale} (KiB per dispatch)")
    head = f"{'share':>6} {'launches':>8} {'avg_us':>8} {'grid':>9} {'rd_MB':>8} {'wr_MB':>7} {'GB/s':>6} {'L2hit':>5}"
    print(head + "".join(f" {c:>14}" for c in extra) + "  kernel")
    pat = re.compile(a.match) if a.match else None
    shown = 0
    for (k, g), (n, us) in order:
        if pat and not pat.search(k):
            continue
        cs = ct.get((k, g))
        if not cs:
            continue
        mean = {c: sum(v) / len(v) for c, v in cs.items()}
        rd = mean.get("FETCH_SIZE", float("nan")) * 1024 * a.fetch_scale / 1e6
        wr = mean.get("WRITE_SIZE", float("nan")) * 1024 * a.write_scale / 1e6
        hit = mean.get("TCC_HIT_sum"), mean.get("TCC_MISS_sum")
        l2 = hit[0] / (hit[0] + hit[1]) if hit[0] is not None and hit[1] is not None and hit[0] + hit[1] > 0 \
            else float("nan")
        avg = us / n
        line = (f"{us / total:6.1%} {n:8d} {avg:8.2f} {g:9d} {rd:8.1f} {wr:7.1f} {(rd + wr) / avg * 1e3:6.0f} "
                f"{l2:5.2f}")
        print(line + "".join(f" {mean.get(c, float('nan')):14.4g}" for c in extra) + "  " + k)
        shown += 1
        if shown >= a.top:
            break
    return 0


if __name__ == "__main__":
    sys.exit(main())
