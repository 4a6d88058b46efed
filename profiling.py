"""Summaries of rocprofv3 output for the fused step (kernel time, counters,
HBM traffic scaled by a copy-kernel calibration).

Usage (on the host that holds the rocprofv3 output directories):

  python profiling.py stats  TRACE_DIR  OUT.md  "command"
  python profiling.py counters OUT.md "command" DIR...
  python profiling.py traffic WORKLOAD FETCH_DIR WRITE_DIR COPY_BYTES

`stats` also lists, from the per-dispatch trace, each kernel's median
duration and its mean over the launches after the first few (the first
launches of a run are slower: cold caches and clocks).

`traffic` scales each counter by (bytes the calibration copy really moved) /
(what the same counter reported for it), and records the result with the
kernel source hash in profiles/traffic.json, which bench.py reads.
"""
from __future__ import annotations

import csv
import glob
import hashlib
import json
import os
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(ROOT, "paper_2602_15883_amd", "csrc")
STEP_KERNEL = "step_kernel"
COPY_KERNEL = "neg_kernel"


def _csvs(d, suffix):
    return sorted(glob.glob(os.path.join(d, "**", "*" + suffix), recursive=True))


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for f in ("ddpinn_kernels.hip", "ddpinn_internal.h"):
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def short(name: str) -> str:
    return name if len(name) < 90 else name[:87] + "..."


def stats(trace_dir: str):
    rows = []
    for path in _csvs(trace_dir, "kernel_stats.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append(r)
    return rows


def dispatch_durations(trace_dir: str):
    """{kernel name: [duration ns of each dispatch, in dispatch order]}"""
    out = defaultdict(list)
    for path in _csvs(trace_dir, "kernel_trace.csv"):
        rows = []
        with open(path) as f:
            for r in csv.DictReader(f):
                rows.append((int(r["Start_Timestamp"]), r["Kernel_Name"],
                             int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for _t, name, d in sorted(rows):
            out[name].append(d)
    return out


def counter_values(d: str):
    """{kernel name: {counter: [values per dispatch]}}"""
    out = defaultdict(lambda: defaultdict(list))
    for path in _csvs(d, "counter_collection.csv"):
        with open(path) as f:
            for r in csv.DictReader(f):
                out[r["Kernel_Name"]][r["Counter_Name"]].append(float(r["Counter_Value"]))
    return out


def _find(kv, sub):
    for k in kv:
        if sub in k:
            return k
    return None


def write_stats_md(trace_dir, out_md, command, skip_first=3):
    rows = stats(trace_dir)
    durs = dispatch_durations(trace_dir)
    lines = [f"# Kernel time: {os.path.basename(out_md)[:-3]}", "",
             "Command (rocprofv3, run from /tmp on the GPU host):", "", "```", command, "```", "",
             f"Median and 'mean after {skip_first}' (the mean over the dispatches after the first "
             f"{skip_first} of each kernel) come from the per-dispatch kernel trace.", "",
             "| Kernel | Calls | Average (us) | Median (us) | Mean after " + str(skip_first) +
             " (us) | Min (us) | Max (us) | Share (%) |",
             "|---|---|---|---|---|---|---|---|"]
    for r in rows:
        d = sorted(durs.get(r["Name"], []))
        tail = durs.get(r["Name"], [])[skip_first:]
        med = f"{d[len(d) // 2] / 1e3:.1f}" if d else "-"
        mt = f"{sum(tail) / len(tail) / 1e3:.1f}" if tail else "-"
        lines.append(f"| `{short(r['Name'])}` | {r['Calls']} | {float(r['AverageNs']) / 1e3:.1f} | "
                     f"{med} | {mt} | "
                     f"{float(r['MinNs']) / 1e3:.1f} | {float(r['MaxNs']) / 1e3:.1f} | "
                     f"{float(r['Percentage']):.2f} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return rows


def write_counters_md(out_md, command, dirs):
    lines = [f"# Counters: {os.path.basename(out_md)[:-3]}", "",
             "Commands (one rocprofv3 --pmc pass each, run from /tmp on the GPU host):", "", "```"]
    lines += [command, "```", "", "Mean per dispatch of the fused step kernel:", "",
              "| Counter | Mean per dispatch |", "|---|---|"]
    merged = {}
    for d in dirs:
        cv = counter_values(d)
        k = _find(cv, STEP_KERNEL)
        if k is None:
            continue
        for c, vals in cv[k].items():
            merged[c] = sum(vals) / len(vals)
    for c in sorted(merged):
        lines.append(f"| {c} | {merged[c]:.6g} |")
    with open(out_md, "w") as f:
        f.write("\n".join(lines) + "\n")
    return merged


def traffic(workload, fetch_dir, write_dir, copy_bytes, out_json=None):
    copy_kib = copy_bytes / 1024.0
    res = {}
    for counter, d in (("FETCH_SIZE", fetch_dir), ("WRITE_SIZE", write_dir)):
        cv = counter_values(d)
        kc = _find(cv, COPY_KERNEL)
        ks = _find(cv, STEP_KERNEL)
        if kc is None or ks is None:
            raise SystemExit(f"{counter}: calibration or step kernel missing in {d}")
        cal = min(cv[kc][counter])          # the copy's reading (KiB)
        scale = copy_kib / cal
        step = sum(cv[ks][counter]) / len(cv[ks][counter])
        res[counter] = {"copy_kib_measured": cal, "scale": scale, "step_kib_raw": step,
                        "step_bytes": step * scale * 1024.0}
    entry = {"bytes_per_launch": res["FETCH_SIZE"]["step_bytes"] + res["WRITE_SIZE"]["step_bytes"],
             "read_bytes": res["FETCH_SIZE"]["step_bytes"], "write_bytes": res["WRITE_SIZE"]["step_bytes"],
             "fetch_scale": res["FETCH_SIZE"]["scale"], "write_scale": res["WRITE_SIZE"]["scale"],
             "kernel_hash": kernel_source_hash()}
    out_json = out_json or os.path.join(ROOT, "profiles", "traffic.json")
    try:
        with open(out_json) as f:
            tab = json.load(f)
    except (OSError, ValueError):
        tab = {}
    tab[workload] = entry
    with open(out_json, "w") as f:
        json.dump(tab, f, indent=1, sort_keys=True)
    return entry


if __name__ == "__main__":
    cmd = sys.argv[1]
    if cmd == "stats":
        for r in write_stats_md(sys.argv[2], sys.argv[3], sys.argv[4]):
            print(r["Name"][:60], r["Calls"], r["AverageNs"])
    elif cmd == "counters":
        print(write_counters_md(sys.argv[2], sys.argv[3], sys.argv[4:]))
    elif cmd == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])))
    else:
        raise SystemExit(__doc__)
