"""Summaries of rocprofv3 output for the kernels of this library.

    python -m paper_1312_2880_amd.profiling stats  <kernel_stats.csv> [title]
    python -m paper_1312_2880_amd.profiling trace  <kernel_trace.csv> [top]
    python -m paper_1312_2880_amd.profiling phases <kernel_trace.csv> <kernel> [marker]
    python -m paper_1312_2880_amd.profiling traffic <fetch_dir> <write_dir> <kernel> <bytes> <hash> [key]

`stats` prints a short markdown table (kernel, calls, average and total
time, share).  `trace` splits the same time by kernel and launch shape
(grid size: one row per level of the hierarchy), with the median duration.
`phases` splits the launches of one kernel (name prefix) at the end of the
last launch of a marker kernel (default the Krylov kernels, k_kry_): in a
bench.py run the launches before it belong to the timed solves, the ones
after it to the per-kernel timing that follows them.  `traffic` combines two `--pmc` runs (FETCH_SIZE, then
WRITE_SIZE; KiB per dispatch) of `bench.py --traffic-probe`: the probe runs
the dominant kernel on cold buffers and a plain device-to-device copy of a
known size; each counter is scaled by (copy bytes / what the counter reads for
the copy), and the per-launch HBM bytes of the kernel are written as JSON.
"""
from __future__ import annotations

import csv
import glob
import json
import os
import sys


def kernel_stats(path: str, title: str = "", top: int = 14) -> str:
    rows = list(csv.DictReader(open(path)))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    out = [f"### {title}" if title else "", "",
           "| share | calls | avg (us) | total (ms) | kernel |", "|---:|---:|---:|---:|---|"]
    for r in rows[:top]:
        name = r["Name"].split("(")[0].replace("void ", "")
        out.append(f"| {100 * float(r['TotalDurationNs']) / total:5.1f}% | {r['Calls']} | "
                   f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['TotalDurationNs']) / 1e6:.2f} | `{name}` |")
    out.append(f"\nall kernels: {total / 1e6:.2f} ms")
    return "\n".join(out)


def kernel_trace(path: str, top: int = 20) -> str:
    rows = list(csv.DictReader(open(path)))
    groups = {}
    for r in rows:
        name = r["Kernel_Name"].split("(")[0].replace("void ", "")
        wx, wy = int(r["Workgroup_Size_X"]), int(r.get("Workgroup_Size_Y", 1) or 1)
        wz = int(r.get("Workgroup_Size_Z", 1) or 1)
        gz = int(r.get("Grid_Size_Z", 1) or 1) // max(wz, 1)
        key = (name, int(r["Grid_Size_X"]) // max(wx, 1), int(r["Grid_Size_Y"]) // max(wy, 1), wx * wy * wz, gz)
        groups.setdefault(key, []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    total = sum(sum(v) for v in groups.values())
    out = ["| share | calls | median (us) | total (ms) | workgroups (x by y by z) | threads | kernel |",
           "|---:|---:|---:|---:|---:|---:|---|"]
    for key, v in sorted(groups.items(), key=lambda kv: -sum(kv[1]))[:top]:
        v.sort()
        out.append(f"| {100 * sum(v) / total:5.1f}% | {len(v)} | {v[len(v) // 2] / 1e3:.2f} | "
                   f"{sum(v) / 1e6:.2f} | {key[1]}x{key[2]}x{key[4]} | {key[3]} | `{key[0]}` |")
    out.append(f"\nall kernels: {total / 1e6:.2f} ms")
    return "\n".join(out)


def kernel_phases(path: str, kernel: str, marker: str = "k_kry_") -> str:
    rows = list(csv.DictReader(open(path)))

    def short(r):
        return r["Kernel_Name"].split("(")[0].replace("void ", "").replace("hmgk::", "")

    end = max(int(r["End_Timestamp"]) for r in rows if short(r).startswith(marker))
    groups = {}
    for r in rows:
        name = short(r)
        if not name.startswith(kernel):
            continue
        phase = "solves" if int(r["Start_Timestamp"]) < end else "kernel timing"
        groups.setdefault((name, phase), []).append(int(r["End_Timestamp"]) - int(r["Start_Timestamp"]))
    out = ["| kernel | phase | launches | mean (us) | median (us) |", "|---|---|---:|---:|---:|"]
    for (name, phase), v in sorted(groups.items()):
        v.sort()
        out.append(f"| `{name}` | {phase} | {len(v)} | {sum(v) / len(v) / 1e3:.2f} | {v[len(v) // 2] / 1e3:.2f} |")
    return "\n".join(out)


def _counter_rows(d: str):
    files = glob.glob(os.path.join(d, "**", "*counter_collection*.csv"), recursive=True)
    rows = []
    for fpath in files:
        rows += list(csv.DictReader(open(fpath)))
    return rows


def _per_dispatch(rows, counter: str, match: str):
    vals = {}
    for r in rows:
        if r.get("Counter_Name") != counter or match not in r.get("Kernel_Name", ""):
            continue
        key = r.get("Dispatch_Id") or r.get("Correlation_Id")
        vals[key] = vals.get(key, 0.0) + float(r["Counter_Value"])
    return list(vals.values())


def traffic(fetch_dir, write_dir, kernel, copy_bytes, src_hash, key):
    fr, wr = _counter_rows(fetch_dir), _counter_rows(write_dir)
    k_fetch = _per_dispatch(fr, "FETCH_SIZE", kernel)
    k_write = _per_dispatch(wr, "WRITE_SIZE", kernel)
    c_fetch = _per_dispatch(fr, "FETCH_SIZE", "copy")
    c_write = _per_dispatch(wr, "WRITE_SIZE", "copy")
    if not (k_fetch and k_write and c_fetch and c_write):
        raise SystemExit("counters missing for the kernel or the copy")
    # the copy reads and writes copy_bytes once: counter (KiB) -> bytes factor
    f_scale = copy_bytes / (max(c_fetch) * 1024.0)
    w_scale = copy_bytes / (max(c_write) * 1024.0)
    fetch = sorted(k_fetch)[len(k_fetch) // 2] * 1024.0 * f_scale
    write = sorted(k_write)[len(k_write) // 2] * 1024.0 * w_scale
    return {key: {"kernel": kernel, "kernel_source_hash": src_hash,
                  "bytes_per_launch": fetch + write, "fetch_bytes": fetch, "write_bytes": write,
                  "fetch_scale": f_scale, "write_scale": w_scale,
                  "dispatches": [len(k_fetch), len(k_write)]}}


if __name__ == "__main__":
    if len(sys.argv) >= 3 and sys.argv[1] == "stats":
        print(kernel_stats(sys.argv[2], sys.argv[3] if len(sys.argv) > 3 else ""))
    elif len(sys.argv) >= 3 and sys.argv[1] == "trace":
        print(kernel_trace(sys.argv[2], int(sys.argv[3]) if len(sys.argv) > 3 else 20))
    elif len(sys.argv) >= 4 and sys.argv[1] == "phases":
        print(kernel_phases(sys.argv[2], sys.argv[3], sys.argv[4] if len(sys.argv) > 4 else "k_kry_"))
    elif len(sys.argv) >= 7 and sys.argv[1] == "traffic":
        key = sys.argv[7] if len(sys.argv) > 7 else f"{sys.argv[4]}:fp64"
        print(json.dumps(traffic(sys.argv[2], sys.argv[3], sys.argv[4], float(sys.argv[5]),
                                 sys.argv[6], key), indent=1))
    else:
        print(__doc__)
        sys.exit(2)
