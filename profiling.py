"""Summaries of rocprofv3 output for the fused step (kernel time, counters,
HBM traffic scaled by a copy-kernel calibration).

Usage (on the host that holds the rocprofv3 output directories):

  python profiling.py stats  TRACE_DIR  OUT.md  "command" [PLAIN_GROUPS]
  python profiling.py counters OUT.md "command" DIR...
  python profiling.py traffic WORKLOAD FETCH_DIR WRITE_DIR COPY_BYTES

`stats` also lists, from the per-dispatch trace, each kernel's median
duration and its mean over the launches after the first few (the first
launches of a run are slower: cold caches and clocks); with PLAIN_GROUPS = n
it also compares the grouped step-kernel launches with the runs of n plain
per-subdomain launches between them.

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


def step_dispatches_by_grid(trace_dir: str):
    """{(step kernel name, grid threads): [duration ns, ...]} in dispatch order"""
    out = defaultdict(list)
    for path in _csvs(trace_dir, "kernel_trace.csv"):
        rows = []
        with open(path) as f:
            for r in csv.DictReader(f):
                if STEP_KERNEL in r["Kernel_Name"]:
                    rows.append((int(r["Start_Timestamp"]), r["Kernel_Name"], int(r["Grid_Size_X"]),
                                 int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
        for _t, name, grid, d in sorted(rows):
            out[(name, grid)].append(d)
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


def write_stats_md(trace_dir, out_md, command, skip_first=3, plain_groups=0):
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
    if plain_groups:
        # grouped launches alternate with runs of plain_groups per-subdomain
        # launches of the same kernel: a dispatch is part of a run when its
        # neighbours are, i.e. split the sequence at the long (grouped) ones
        seq_all = []
        for path in _csvs(trace_dir, "kernel_trace.csv"):
            with open(path) as f:
                seq_all += [(int(r["Start_Timestamp"]), int(r["End_Timestamp"]))
                            for r in csv.DictReader(f) if STEP_KERNEL in r["Kernel_Name"]]
        seq_all.sort()
        durs = [e - b for b, e in seq_all]
        cut = (max(durs) + min(durs)) / 2
        runs, cur = [], []
        grouped = []
        for d in durs:
            if d > cut:
                if len(cur) == plain_groups:
                    runs.append(cur)
                cur = []
                grouped.append(d)
            else:
                cur.append(d)
        if len(cur) == plain_groups:
            runs.append(cur)
        sums = sorted(sum(r) for r in runs)
        gs = sorted(grouped)
        if sums and gs:
            lines += ["", f"Grouped launch vs {plain_groups} plain per-subdomain launches (the step kernel's "
                      f"dispatches split at {cut / 1e3:.0f} us; plain launches summed per step, kernel "
                      "execution only):", "",
                      "| Launch | Steps | Median (us) |", "|---|---|---|",
                      f"| one grouped launch | {len(gs)} | {gs[len(gs) // 2] / 1e3:.1f} |",
                      f"| {plain_groups} plain launches (sum) | {len(sums)} | {sums[len(sums) // 2] / 1e3:.1f} |",
                      f"| ratio plain / grouped | | {sums[len(sums) // 2] / gs[len(gs) // 2]:.3f} |"]
    by_grid = step_dispatches_by_grid(trace_dir)
    if len(by_grid) > 1:
        lines += ["", "Step-kernel dispatches by grid size (workgroups x threads):", "",
                  "| Kernel | Grid threads | Calls | Median (us) | Mean after " + str(skip_first) + " (us) |",
                  "|---|---|---|---|---|"]
        for (name, grid), d in sorted(by_grid.items(), key=lambda kv: -kv[0][1]):
            ds = sorted(d)
            tail = d[skip_first:]
            mt = f"{sum(tail) / len(tail) / 1e3:.1f}" if tail else "-"
            lines.append(f"| `{short(name)}` | {grid} | {len(d)} | {ds[len(ds) // 2] / 1e3:.1f} | {mt} |")
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
        pg = int(sys.argv[5]) if len(sys.argv) > 5 else 0
        for r in write_stats_md(sys.argv[2], sys.argv[3], sys.argv[4], plain_groups=pg):
            print(r["Name"][:60], r["Calls"], r["AverageNs"])
    elif cmd == "counters":
        print(write_counters_md(sys.argv[2], sys.argv[3], sys.argv[4:]))
    elif cmd == "traffic":
        print(traffic(sys.argv[2], sys.argv[3], sys.argv[4], int(sys.argv[5])))
    else:
        raise SystemExit(__doc__)
