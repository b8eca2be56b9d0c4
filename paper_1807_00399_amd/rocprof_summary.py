"""Summarise rocprofv3 CSV output into the short files kept under profiles/.

    python -m paper_1807_00399_amd.rocprof_summary stats  <kernel_stats.csv> <out.txt> "<command>"
    python -m paper_1807_00399_amd.rocprof_summary traffic <kernel-regex> <fetch.csv> <write.csv> \\
           <copy_fetch.csv> <copy_write.csv> <copy_bytes> <launches_per_step> <out.json> "<command>"

    python -m paper_1807_00399_amd.rocprof_summary valu <kernel-regex> <sq.csv> <launches_per_call> <out.json> "<command>"

`stats` keeps the per-kernel call count, total and average duration.
`traffic` turns FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of the matching
kernel into bytes per launch, each scaled by the ratio between the known
bytes of a plain copy kernel and what the same counter reported for it.
`valu` turns SQ_WAVES, SQ_INSTS_VALU and SQ_INSTS_VMEM_RD of each matching
dispatch into instructions per wave and the share of the chip's vector issue
slots the dispatch used: a wave64 vector instruction occupies a 16-lane SIMD
for 4 cycles, and MI355X has 256 CUs x 4 SIMDs at 2.4 GHz, so the nominal share is
4 * SQ_INSTS_VALU / (1024 * 2.4e9 * duration) (nominal: some vector instructions
issue in fewer cycles, so it can exceed 1).
"""
from __future__ import annotations

import csv
import json
import re
import statistics
import sys


def _demangle(name: str) -> str:
    """Itanium-mangled kernel names (some ROCm versions report them so) in
    readable form, through c++filt when it is installed."""
    if not name.startswith("_Z"):
        return name
    import subprocess
    try:
        r = subprocess.run(["c++filt", name], capture_output=True, text=True, timeout=10)
        out = r.stdout.strip()
        if out and out != name:
            return out
    except (OSError, subprocess.SubprocessError):
        pass
    # c++filt without support for some argument types: the nested name's
    # identifiers (<length><name> ... up to E, or I for template arguments)
    if not name.startswith("_ZN"):
        return name
    ids, pos = [], 3
    while pos < len(name) and name[pos].isdigit():
        k = pos
        while name[k].isdigit():
            k += 1
        n = int(name[pos:k])
        ids.append(name[k:k + n])
        pos = k + n
    ids = [i for i in ids if not i.startswith("_GLOBAL__N")]
    if not ids:
        return name
    targs = ""
    if name[pos:pos + 1] == "I":
        # template arguments that are literals (L<type><value>E, as in
        # ILb1E or ILi64ELi8E) are spelled out; anything else stays "..."
        m = re.match(r"I((?:L[bijl]n?\d+E)+)E", name[pos:])
        if m:
            vals = []
            for t, v in re.findall(r"L([bijl])(n?\d+)E", m.group(1)):
                v = v.replace("n", "-")
                vals.append(("true" if v == "1" else "false") if t == "b" else v)
            targs = "<" + ", ".join(vals) + ">"
        else:
            targs = "<...>"
    return "::".join(ids) + targs + "("


def _short(name: str) -> str:
    name = _demangle(name).replace("(anonymous namespace)::", "").replace("void ", "")
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
    from bench import kernel_digest, kernel_tag_of
    res["kernel_digest"] = kernel_digest(kernel_tag_of(regex))
    json.dump(res, open(out, "w"), indent=1)


def valu(regex, sq_csv, per_call, out, command):
    per = {}
    for r in csv.DictReader(open(sq_csv)):
        if not re.search(regex, r["Kernel_Name"]):
            continue
        d = per.setdefault(int(r["Dispatch_Id"]), {"ns": float(r["End_Timestamp"]) - float(r["Start_Timestamp"])})
        d[r["Counter_Name"]] = d.get(r["Counter_Name"], 0.0) + float(r["Counter_Value"])
    rows = []
    for k in sorted(per):
        d = per[k]
        w = d["SQ_WAVES"]
        rows.append({"dispatch": k, "us": d["ns"] / 1e3, "waves": w,
                     "valu_per_wave": d["SQ_INSTS_VALU"] / w, "vmem_rd_per_wave": d["SQ_INSTS_VMEM_RD"] / w,
                     "valu_issue_share_nominal": 4.0 * d["SQ_INSTS_VALU"] / (1024 * 2.4e9 * d["ns"] * 1e-9)})
    res = {"kernel_regex": regex, "command": command, "dispatches": len(rows),
           "valu_issue_share_nominal_time_weighted": sum(r["valu_issue_share_nominal"] * r["us"] for r in rows) /
           sum(r["us"] for r in rows),
           "first_call": [{"us": round(r["us"], 1), "valu_per_wave": round(r["valu_per_wave"]),
                           "vmem_rd_per_wave": round(r["vmem_rd_per_wave"], 1),
                           "valu_issue_share_nominal": round(r["valu_issue_share_nominal"], 3)}
                          for r in rows[:int(per_call)]]}
    from bench import kernel_digest, kernel_tag_of
    res["kernel_digest"] = kernel_digest(kernel_tag_of(regex))
    json.dump(res, open(out, "w"), indent=1)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        stats(*sys.argv[2:5])
    elif sys.argv[1] == "traffic":
        traffic(*sys.argv[2:11])
    elif sys.argv[1] == "valu":
        valu(*sys.argv[2:7])
    else:
        raise SystemExit(__doc__)
