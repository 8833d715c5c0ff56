"""Summarise rocprofv3 result databases as short text.

    python -m paper_1806_10889_amd.profsummary DB [DB ...]

For a kernel-trace database: per kernel, calls, total and average duration
(microseconds) and share of GPU time.  For a counter-collection database: per
kernel, the number of dispatches, their average duration in that same run
(when it was collected with --kernel-trace) and the per-dispatch average of
every collected counter.
"""
from __future__ import annotations

import collections
import sqlite3
import sys


def summarise(path: str) -> str:
    con = sqlite3.connect(path)
    tables = {r[0] for r in con.execute("select name from sqlite_master")}
    out = [f"# {path}"]
    has_counters = False
    if "counters_collection" in tables:
        agg = collections.defaultdict(lambda: collections.defaultdict(float))
        disp = collections.defaultdict(set)
        for kn, cn, v, did in con.execute(
                "select kernel_name, counter_name, value, dispatch_id from counters_collection"):
            k = kn.split("(")[0]
            agg[k][cn] += v
            disp[k].add(did)
        if agg:
            has_counters = True
            dur = {}
            if "kernels" in tables:
                for did, d in con.execute("select dispatch_id, duration from kernels"):
                    dur[did] = d
            out.append("kernel | dispatches | average_us (same run) | per-dispatch average of each counter")
            for k in sorted(agg, key=lambda k: -len(disp[k])):
                n = len(disp[k])
                ds = [dur[d] for d in disp[k] if d in dur]
                avg_us = f"{sum(ds) / len(ds) / 1e3:.3f}" if ds else "-"
                vals = ", ".join(f"{c}={agg[k][c] / n:.6g}" for c in sorted(agg[k]))
                out.append(f"{k} | {n} | {avg_us} | {vals}")
    if "top_kernels" in tables and not has_counters:
        out.append("kernel | calls | total_us | average_us | percent")
        for name, calls, tot, avg, pctg in con.execute(
                "select name, total_calls, total_duration, average, percentage from top_kernels"):
            out.append(f"{name.split('(')[0]} | {calls} | {tot:.1f} | {avg:.3f} | {pctg:.2f}")
    return "\n".join(out)


def main(argv):
    for p in argv:
        print(summarise(p))
        print()


if __name__ == "__main__":
    main(sys.argv[1:])
