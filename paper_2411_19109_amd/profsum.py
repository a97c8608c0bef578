"""Condense rocprofv3 CSV output into short per-kernel text summaries.

    python -m paper_2411_19109_amd.profsum stats DIR   # --kernel-trace --stats run
    python -m paper_2411_19109_amd.profsum pmc DIR     # --pmc COUNTER run

``stats`` prints, per kernel, the call count and the average / total device
time from the *_kernel_stats.csv file.  ``pmc`` prints, per kernel, the number
of dispatches and the mean and largest counter value per dispatch from the
*_counter_collection.csv file (FETCH_SIZE / WRITE_SIZE are in KiB).
"""
from __future__ import annotations

import collections
import csv
import glob
import os
import re
import sys


def _short(name: str) -> str:
    m = re.search(r"(k_\w+)<([^>]*)>", name)
    if m:
        return f"{m.group(1)}<{m.group(2)}>"
    return name.split("(")[0][:60]


def stats(d: str) -> str:
    f = glob.glob(os.path.join(d, "**", "*kernel_stats.csv"), recursive=True)[0]
    rows = list(csv.DictReader(open(f)))
    out = ["kernel | calls | avg_us | min_us | max_us | total_ms | percent"]
    for r in rows:
        out.append(f"{_short(r['Name'])} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.3f} | "
                   f"{float(r['MinNs']) / 1e3:.3f} | {float(r['MaxNs']) / 1e3:.3f} | "
                   f"{float(r['TotalDurationNs']) / 1e6:.2f} | {float(r['Percentage']):.2f}")
    return "\n".join(out)


def pmc(d: str) -> str:
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    agg = collections.defaultdict(list)
    with open(f) as fh:
        for r in csv.DictReader(fh):
            agg[(_short(r["Kernel_Name"]), r["Counter_Name"])].append(float(r["Counter_Value"]))
    out = ["kernel | counter | dispatches | mean_per_dispatch | max_per_dispatch"]
    for (k, c), v in sorted(agg.items()):
        out.append(f"{k} | {c} | {len(v)} | {sum(v) / len(v):.3f} | {max(v):.3f}")
    return "\n".join(out)


if __name__ == "__main__":
    mode, d = sys.argv[1], sys.argv[2]
    print(stats(d) if mode == "stats" else pmc(d))
