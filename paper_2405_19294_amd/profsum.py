"""Summaries of rocprofv3 output for the hopping kernel.

``python -m paper_2405_19294_amd.profsum STATS_CSV FETCH_CSV WRITE_CSV OUT_PREFIX``
reads a ``--kernel-trace --stats`` kernel_stats.csv and two ``--pmc``
counter_collection.csv files (FETCH_SIZE and WRITE_SIZE runs of the same
command) and writes ``OUT_PREFIX.md`` (a short table) and ``OUT_PREFIX.json``
(HBM bytes per launch of each hopping-kernel instance).

Counter calibration: both counters are in KiB per dispatch.  They are scaled
by what they read for a device-to-device copy of known size in the same run
(the 1 GiB copy ``bench.py`` performs after its timed steps): on MI355X
FETCH_SIZE reports half of the bytes that copy reads and WRITE_SIZE reports
exactly the bytes it writes.  The JSON carries the hash of the kernel sources
the counters were taken with; ``bench.py`` reports the traffic only while the
current sources hash to the same value.
"""

from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
KERNEL_SOURCES = ("csrc/hop_impl.h", "csrc/hrw_internal.h", "csrc/kernels.h")
COPY_BYTES = 1 << 30


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for rel in KERNEL_SOURCES:
        with open(os.path.join(HERE, rel), "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def _per_kernel(path):
    d = collections.defaultdict(list)
    for r in csv.DictReader(open(path)):
        d[r["Kernel_Name"]].append(float(r["Counter_Value"]) * 1024.0)
    return d


def _copy_factor(d, expect):
    """Scale factor from the 1 GiB copies (largest copyBuffer dispatches)."""
    vals = [v for k, vs in d.items() if "copyBuffer" in k for v in vs]
    big = [v for v in vals if v > expect / 4]
    if not big:
        return None
    return expect / statistics.median(big)


def summarize(stats_csv, fetch_csv, write_csv, out_prefix, command=""):
    fetch = _per_kernel(fetch_csv)
    write = _per_kernel(write_csv)
    ff = _copy_factor(fetch, COPY_BYTES)
    wf = _copy_factor(write, COPY_BYTES)
    stats = list(csv.DictReader(open(stats_csv))) if stats_csv else []
    avg_us = {r["Name"]: float(r["AverageNs"]) / 1e3 for r in stats}
    calls = {r["Name"]: int(r["Calls"]) for r in stats}
    rows = []
    for name in sorted(fetch, key=lambda k: -sum(fetch[k])):
        if not any(k in name for k in ("hop_kernel", "hop_mrhs_kernel", "hop_su3_kernel", "hop_fused_kernel")):
            continue
        fb = statistics.mean(fetch[name]) * (ff or 1.0)
        wb = statistics.mean(write.get(name, [0.0])) * (wf or 1.0)
        rows.append({"kernel": name, "fetch_bytes": fb, "write_bytes": wb, "traffic_bytes": fb + wb,
                     "avg_us": avg_us.get(name), "calls": calls.get(name)})
    rec = {"source_hash": kernel_source_hash(), "fetch_factor": ff, "write_factor": wf, "kernels": rows,
           "command": command}
    with open(out_prefix + ".json", "w") as f:
        json.dump(rec, f, indent=1)
    lines = ["# HBM traffic of the hopping kernels (rocprofv3 --pmc FETCH_SIZE / WRITE_SIZE)", ""]
    if command:
        lines += ["Command (one run per counter):", "", "```", command, "```", ""]
    lines += [f"Calibration against a 1 GiB device copy in the same run: FETCH_SIZE x {ff:.3f}, "
              f"WRITE_SIZE x {wf:.3f}.", "", "| kernel | fetch MB | write MB | traffic MB |", "|---|---|---|---|"]
    for r in rows:
        lines.append(f"| `{r['kernel'].replace('void ', '').split('(')[0]}` | {r['fetch_bytes'] / 1e6:.1f} | "
                     f"{r['write_bytes'] / 1e6:.1f} | {r['traffic_bytes'] / 1e6:.1f} |")
    lines += ["", f"Kernel source hash: {rec['source_hash']}"]
    with open(out_prefix + ".md", "w") as f:
        f.write("\n".join(lines) + "\n")
    return rec


def stats_table(stats_csv, out_md, title, command, top=14):
    rows = list(csv.DictReader(open(stats_csv)))
    lines = [f"# {title}", "", "Command:", "", "```", command, "```", "",
             "| kernel | calls | avg us | min us | max us | share |", "|---|---|---|---|---|---|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"]))[:top]:
        name = r["Name"].replace("void ", "").split("(")[0]
        lines.append(f"| `{name}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.1f}% |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")


def traffic_for(kernel_substr: str, path: str):
    """Traffic bytes per launch recorded for a kernel, or None when the record is
    missing or was taken with different kernel sources."""
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_hash") != kernel_source_hash():
        return None
    for r in rec.get("kernels", []):
        if kernel_substr in r["kernel"]:
            return r["traffic_bytes"]
    return None


if __name__ == "__main__":
    summarize(sys.argv[1], sys.argv[2], sys.argv[3], sys.argv[4], " ".join(sys.argv[5:]))
