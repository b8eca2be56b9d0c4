"""Summarise rocprofv3 CSV output into the short files kept under profiles/.

    python -m paper_1807_00399_amd.rocprof_summary stats  <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_1807_00399_amd.rocprof_summary traffic <kernel-regex> <fetch.csv> <write.csv> \\
           <copy_fetch.csv> <copy_write.csv> <copy_bytes> <launches_per_step> <out.json> "<command>"

`stats` keeps the per-kernel call count, total and average duration.
`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the matching
kernel into bytes per launch, each scaled by the ratio between the known
bytes of a plain copy kernel and what the same counter reported for it.
"""
from __future__ import annotations

import csv
import json
import re
import statistics
import sys


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "").replace("void ", "")
    return name.split("(")[0]


def stats(path: str, out: str, command: str):
    rows = list(csv.DictReader(open(path)))
    lines = [f"# rocprofv3 --kernel-trace --stats summary", f"# command: {command}",
             f"{'calls':>7} {'total_us':>12} {'avg_us':>10} {'min_us':>10} {'max_us':>10} {'pct':>6}  kernel"]
    for r in rows:
        calls = int(r["Calls"])
        tot = float(r["TotalDurationNs"]) / 1e3
        lines.append(f"{calls:>7} {tot:>12.1f} {float(r['AverageNs']) / 1e3:>10.2f} "
                     f"{float(r['MinNs']) / 1e3:>10.2f} {float(r['MaxNs']) / 1e3:>10.2f} "
                     f"{float(r['Percentage']):>6.2f}  {_short(r['Name'])}")
    open(out, "w").write("\n".join(lines) + "\n")


def _counter(path: str, regex: str, counter: str):
    vals = []
    for r in csv.DictReader(open(path)):
        if r["Counter_Name"] == counter and re.search(regex, r["Kernel_Name"]):
            vals.append(float(r["Counter_Value"]))
    return vals


def traffic(regex, fetch_csv, write_csv, copy_fetch_csv, copy_write_csv, copy_bytes, per_step, out, command):
    copy_bytes = float(copy_bytes)
    cf = statistics.median(_counter(copy_fetch_csv, "copy", "FETCH_SIZE")) * 1024.0
    cw = statistics.median(_counter(copy_write_csv, "copy", "WRITE_SIZE")) * 1024.0
    f = [v * 1024.0 * copy_bytes / cf for v in _counter(fetch_csv, regex, "FETCH_SIZE")]
    w = [v * 1024.0 * copy_bytes / cw for v in _counter(write_csv, regex, "WRITE_SIZE")]
    res = {
        "kernel_regex": regex, "command": command,
        "copy_calibration": {"bytes": copy_bytes, "fetch_counter_bytes": cf, "write_counter_bytes": cw,
                             "fetch_scale": copy_bytes / cf, "write_scale": copy_bytes / cw},
        "launches": len(f), "launches_per_step": int(per_step),
        "fetch_bytes_per_launch_mean": statistics.mean(f), "write_bytes_per_launch_mean": statistics.mean(w),
        "fetch_bytes_per_launch_median": statistics.median(f),
        "write_bytes_per_launch_median": statistics.median(w),
        "hbm_bytes_per_launch": statistics.mean(f) + statistics.mean(w),
    }
    from bench import kernel_digest
    res["kernel_digest"] = kernel_digest()
    json.dump(res, open(out, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:11])
    else:
        raise SystemExit(__doc__)
