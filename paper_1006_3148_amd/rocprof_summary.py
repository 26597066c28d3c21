"""Summarise rocprofv3 result databases (kernel durations and PMC counters).

Usage:
  python -m paper_1006_3148_amd.rocprof_summary trace <results.db>
  python -m paper_1006_3148_amd.rocprof_summary pmc <results.db> [...]

``trace`` prints per-kernel dispatch count and mean/min/max duration (us);
``pmc`` prints, per kernel and counter, the mean over dispatches of the
counter summed over its dimensions (FETCH_SIZE / WRITE_SIZE are in KiB).
"""

from __future__ import annotations

import collections
import sqlite3
import sys


def _short(name: str) -> str:
    name = name.replace("jacobi_impl::(anonymous namespace)::", "")
    return name[:90]


def trace(path: str) -> str:
    con = sqlite3.connect(path)
    rows = con.execute("select name, duration from kernels").fetchall()
    agg = collections.defaultdict(list)
    for n, d in rows:
        agg[_short(n)].append(d / 1e3)
    out = ["| kernel | calls | mean us | min us | max us | total ms |",
           "|---|---|---|---|---|---|"]
    for n, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        out.append("| %s | %d | %.2f | %.2f | %.2f | %.3f |" % (
            n, len(v), sum(v) / len(v), min(v), max(v), sum(v) / 1e3))
    return "\n".join(out)


def pmc(path: str) -> str:
    con = sqlite3.connect(path)
    rows = con.execute("select kernel_name, counter_name, value, dispatch_id "
                       "from counters_collection").fetchall()
    per = collections.defaultdict(lambda: collections.defaultdict(float))
    for kn, cn, v, d in rows:
        per[(_short(kn), cn)][d] += v
    out = ["| kernel | counter | dispatches | mean per dispatch |",
           "|---|---|---|---|"]
    for (kn, cn), dd in sorted(per.items()):
        vals = list(dd.values())
        out.append("| %s | %s | %d | %.6g |" % (kn, cn, len(vals),
                                               sum(vals) / len(vals)))
    return "\n".join(out)


if __name__ == "__main__":
    mode = sys.argv[1]
    for p in sys.argv[2:]:
        print("##", p)
        print(trace(p) if mode == "trace" else pmc(p))
