"""Condense rocprofv3 CSV output into short per-kernel text summaries.

    python -m paper_2411_19109_amd.profsum stats DIR   # --kernel-trace --stats run
    python -m paper_2411_19109_amd.profsum pmc DIR     # --pmc COUNTER run
    python -m paper_2411_19109_amd.profsum traffic FETCH_DIR WRITE_DIR [LAUNCH_FILE|-] [SOURCE]  # HBM bytes per dispatch
    python -m paper_2411_19109_amd.profsum gaps DIR    # --kernel-trace run: device busy vs idle time

``stats`` prints, per kernel, the call count and the average / total device
time from the *_kernel_stats.csv file.  ``pmc`` prints, per kernel, the number
of dispatches and the mean and largest counter value per dispatch from the
*_counter_collection.csv file (FETCH_SIZE / WRITE_SIZE are in KiB).
``gaps`` reads the *_kernel_trace.csv file and splits the span of the solver
kernels into time with at least one kernel running and idle time between them.
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


def _per_kernel(d: str, counter: str):
    f = glob.glob(os.path.join(d, "**", "*counter_collection.csv"), recursive=True)[0]
    agg = collections.defaultdict(list)
    with open(f) as fh:
        for r in csv.DictReader(fh):
            if r["Counter_Name"] == counter:
                agg[_short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return agg


def gaps(d: str) -> str:
    """Device busy time (the union of all kernel intervals) against the idle
    time between kernels, over the span from the first to the last solver
    kernel (names k_*) of the trace."""
    f = glob.glob(os.path.join(d, "**", "*kernel_trace.csv"), recursive=True)[0]
    iv = []
    with open(f) as fh:
        for r in csv.DictReader(fh):
            iv.append((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), _short(r["Kernel_Name"])))
    iv.sort()
    solver = [i for i, v in enumerate(iv) if v[2].startswith("k_")]
    iv = iv[solver[0]:solver[-1] + 1]
    busy, idle, end, n_gap = 0, 0, iv[0][0], 0
    for s0, s1, _ in iv:
        if s0 > end:
            idle += s0 - end
            n_gap += 1
        busy += max(0, s1 - max(s0, end))
        end = max(end, s1)
    span = end - iv[0][0]
    return (f"kernels {len(iv)} | span_ms {span / 1e6:.2f} | busy_ms {busy / 1e6:.2f} | idle_ms {idle / 1e6:.2f} | "
            f"idle_gaps {n_gap} | mean_gap_us {idle / max(n_gap, 1) / 1e3:.2f} | "
            f"busy_per_kernel_us {busy / len(iv) / 1e3:.2f}")


def kernel_source_hash(source: str = "llg_kernels.hip") -> str:
    """sha256 of the kernel source the counters belong to."""
    import hashlib
    src = os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", source)
    return hashlib.sha256(open(src, "rb").read()).hexdigest()


def traffic(fetch_dir: str, write_dir: str, launch=None, copy_bytes: int = 1 << 28,
            source: str = "llg_kernels.hip") -> str:
    """HBM bytes per dispatch of the solver kernels from a FETCH_SIZE run and a
    WRITE_SIZE run (KiB per dispatch), each scaled by the factor that maps the
    same counter on a plain device copy of copy_bytes (the largest copy
    dispatch of the run) to its true size.  One JSON line."""
    import json
    fe, wr = _per_kernel(fetch_dir, "FETCH_SIZE"), _per_kernel(write_dir, "WRITE_SIZE")
    cal = "__amd_rocclr_copyBuffer"
    kf = copy_bytes / (max(fe[cal]) * 1024.0)
    kw = copy_bytes / (max(wr[cal]) * 1024.0)
    out = {"kernel_source_sha256": kernel_source_hash(source), "source": source, "launch": launch,
           "copy_bytes": copy_bytes,
           "fetch_scale": kf, "write_scale": kw, "kernels": {}}
    for k in sorted(set(fe) & set(wr)):
        if not k.startswith("k_"):
            continue
        f = sum(fe[k]) / len(fe[k]) * 1024.0 * kf
        w = sum(wr[k]) / len(wr[k]) * 1024.0 * kw
        out["kernels"][k] = {"dispatches": len(fe[k]), "fetch_bytes": f, "write_bytes": w, "hbm_bytes": f + w}
    return json.dumps(out)


if __name__ == "__main__":
    mode = sys.argv[1]
    if mode == "traffic":
        # traffic FETCH_DIR WRITE_DIR [LAUNCH_FILE or -] [KERNEL_SOURCE]
        lf = sys.argv[4] if len(sys.argv) > 4 else "-"
        launch = [int(v) for v in open(lf).read().split()] if lf != "-" else None
        print(traffic(sys.argv[2], sys.argv[3], launch, source=sys.argv[5] if len(sys.argv) > 5 else "llg_kernels.hip"))
    else:
        d = sys.argv[2]
        print({"stats": stats, "pmc": pmc, "gaps": gaps}[mode](d))
