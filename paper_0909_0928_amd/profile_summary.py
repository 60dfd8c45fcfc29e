"""Condense rocprofv3 output into the short text summaries kept under profiles/.

    python -m paper_0909_0928_amd.profile_summary trace  --dir D --command "..." --out profiles/X.md
    python -m paper_0909_0928_amd.profile_summary traffic --fetch D1 --write D2 --fetch-copy D3 --write-copy D4 \
        --kernel force --command "..." --out profiles/force_traffic.json

`trace` reads <dir>/*_kernel_stats.csv and *_kernel_trace.csv written by
`rocprofv3 --kernel-trace --stats --output-format csv`.  `traffic` reads the
*_counter_collection.csv files of `rocprofv3 --pmc FETCH_SIZE` and `--pmc
WRITE_SIZE` runs of the benchmark and of `bench.py --copy-probe` (a plain
device copy of 256 MiB), scales each counter by bytes-known / counter-reading
of the copy, and records the per-launch HBM bytes of one kernel together with
a SHA-256 of the kernel sources, so a later benchmark can tell whether the
numbers still describe the code it runs.
"""
from __future__ import annotations

import argparse
import collections
import csv
import glob
import hashlib
import json
import os
import re

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
COPY_BYTES = 256 * 1024 * 1024  # bench.py --copy-probe: one read and one write of this many bytes per copy

# Library kernel name -> source files whose text defines it (for the fingerprint).
KERNEL_SOURCES = {
    "force": ["k_force.hip", "device_common.h", "dir_internal.h"],
    "smooth_yz": ["k_smooth.hip", "device_common.h", "dir_internal.h"],
    "warp": ["k_pyramid.hip", "device_common.h", "dir_internal.h"],
    "warp_pair": ["k_pyramid.hip", "device_common.h", "dir_internal.h"],
}
# Library kernel name -> device symbol stem in rocprofv3 output.
KERNEL_SYMBOL = {"force": "k_force_x", "smooth_yz": "k_smooth_yz", "warp": "k_warp_diff", "warp_pair": "k_warp_pair"}


def source_fingerprint(kernel: str) -> str:
    h = hashlib.sha256()
    for f in KERNEL_SOURCES[kernel]:
        with open(os.path.join(CSRC, f), "rb") as fh:
            h.update(f.encode() + b"\0" + fh.read())
    return h.hexdigest()


def _short(name: str) -> str:
    n = name.replace("dir::(anonymous namespace)::", "").replace("void ", "")
    return re.sub(r"\(.*", "", n)


def _one(pattern: str) -> str:
    hits = sorted(glob.glob(pattern))
    if not hits:
        raise SystemExit(f"no file matches {pattern}")
    return hits[0]


def trace_summary(d: str, command: str, out: str) -> None:
    stats = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_stats.csv")))))
    trace = list(csv.DictReader(open(_one(os.path.join(d, "*kernel_trace.csv")))))
    per = collections.defaultdict(list)
    solo = collections.defaultdict(list)   # launches during which no other kernel ran
    recs = sorted(((int(r["Start_Timestamp"]), int(r["End_Timestamp"]), r) for r in trace), key=lambda t: t[0])
    max_end = -1
    for i, (t0, t1, r) in enumerate(recs):
        g = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        k = _short(r["Kernel_Name"])
        us = (t1 - t0) / 1e3
        per[(k, g)].append(us)
        alone = max_end <= t0 and (i + 1 == len(recs) or recs[i + 1][0] >= t1)
        if alone:
            solo[(re.sub(r"<.*", "", k), g)].append(us)
        max_end = max(max_end, t1)
    lines = ["# rocprofv3 kernel trace summary", "", "Command (repository root, on one MI355X):", "",
             "```", command, "```", "",
             "## Per kernel (rocprofv3 --stats)", "",
             "| kernel | calls | total ms | average us | % |", "|---|---|---|---|---|"]
    for r in stats[:25]:
        lines.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {float(r['TotalDurationNs']) / 1e6:.2f} | "
                     f"{float(r['AverageNs']) / 1e3:.2f} | {float(r['Percentage']):.1f} |")
    agg = collections.defaultdict(list)
    for (k, g), v in per.items():
        agg[re.sub(r"<.*", "", k)] += v
    lines += ["", "## Per library kernel, all instantiations and sizes (from the kernel trace)", "",
              "| kernel | calls | average us | total ms |", "|---|---|---|---|"]
    for k, v in sorted(agg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / 1e3:.2f} |")
    lines += ["", "## Launches that ran alone on the device (no other kernel overlapping), per library kernel",
              "", "| kernel | grid threads | calls | average us |", "|---|---|---|---|"]
    sagg = collections.defaultdict(list)
    for (k, g), v in solo.items():
        sagg[k] += v
    for k, v in sorted(sagg.items(), key=lambda kv: -sum(kv[1])):
        lines.append(f"| `{k}` | all | {len(v)} | {sum(v) / len(v):.2f} |")
        for (k2, g), v2 in sorted(solo.items(), key=lambda kv: -kv[0][1]):
            if k2 == k:
                lines.append(f"| `{k}` | {g} | {len(v2)} | {sum(v2) / len(v2):.2f} |")
    # steps end with the inverse-consistent registration's composition
    ends = [i for i, (_, _, r) in enumerate(recs) if "k_compose" in r["Kernel_Name"]]
    if ends:
        lines += ["", "## Device time per step (launches up to each composition; the step's first launches wait "
                  "for the host)", "",
                  "| step | launches | span ms | kernels ms | idle ms | idle, excluding the wait for the first "
                  "launch and the copy-backs, ms |", "|---|---|---|---|---|---|"]
        lo = 0
        for n, hi in enumerate(ends):
            seg = recs[lo:hi + 1]
            span = (seg[-1][1] - seg[0][0]) / 1e6
            busy = sum(t1 - t0 for t0, t1, _ in seg) / 1e6
            idle_k = 0.0
            for (a0, a1, _), (b0, b1, rb) in zip(seg, seg[1:]):
                if "copyBuffer" not in rb["Kernel_Name"] and "copyBuffer" not in _["Kernel_Name"]:
                    idle_k += max(b0 - a1, 0) / 1e6
            lines.append(f"| {n} | {len(seg)} | {span:.2f} | {busy:.2f} | {span - busy:.2f} | {idle_k:.2f} |")
            lo = hi + 1
    lines += ["", "## Per kernel and grid size (from the kernel trace)", "",
              "| kernel | grid threads | calls | average us | total ms |", "|---|---|---|---|---|"]
    for (k, g), v in sorted(per.items(), key=lambda kv: -sum(kv[1]))[:30]:
        lines.append(f"| `{k}` | {g} | {len(v)} | {sum(v) / len(v):.2f} | {sum(v) / 1e3:.2f} |")
    with open(out, "w") as fh:
        fh.write("\n".join(lines) + "\n")


def _counter_rows(d: str):
    return list(csv.DictReader(open(_one(os.path.join(d, "*counter_collection.csv")))))


def _copy_factor(d: str, expected_kib: float) -> float:
    vals = [float(r["Counter_Value"]) for r in _counter_rows(d) if "copyBuffer" in r["Kernel_Name"]]
    if not vals:
        raise SystemExit(f"no copy kernel in {d}")
    return expected_kib / (sum(vals) / len(vals))


def traffic_summary(fetch: str, write: str, fetch_copy: str, write_copy: str, kernel: str, command: str,
                    out: str, largest_grid: bool = False) -> dict:
    """largest_grid: count only the kernel's launches of the largest grid (the
    finest level of the largest volume in the run)."""
    kib = COPY_BYTES / 1024.0
    ff = _copy_factor(fetch_copy, kib)
    wf = _copy_factor(write_copy, kib)
    sym = KERNEL_SYMBOL[kernel]

    def mean_kib(d):
        rows = [r for r in _counter_rows(d) if _short(r["Kernel_Name"]).startswith(sym)]
        if largest_grid:
            g = max(int(r["Grid_Size"]) for r in rows)
            rows = [r for r in rows if int(r["Grid_Size"]) == g]
        v = [float(r["Counter_Value"]) for r in rows]
        return sum(v) / len(v), len(v)

    fk, nf = mean_kib(fetch)
    wk, nw = mean_kib(write)
    res = {
        "kernel": kernel, "symbol": sym, "source_sha256": source_fingerprint(kernel),
        "launches_counted": {"fetch": nf, "write": nw},
        "fetch_factor": ff, "write_factor": wf,
        "fetch_bytes_per_launch": fk * 1024.0 * ff, "write_bytes_per_launch": wk * 1024.0 * wf,
        "command": command,
    }
    res["traffic_bytes_per_launch"] = res["fetch_bytes_per_launch"] + res["write_bytes_per_launch"]
    with open(out, "w") as fh:
        json.dump(res, fh, indent=1)
        fh.write("\n")
    return res


def main():
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("trace")
    t.add_argument("--dir", required=True)
    t.add_argument("--command", required=True)
    t.add_argument("--out", required=True)
    c = sub.add_parser("traffic")
    for k in ("fetch", "write", "fetch-copy", "write-copy"):
        c.add_argument("--" + k, required=True)
    c.add_argument("--kernel", default="force")
    c.add_argument("--command", required=True)
    c.add_argument("--out", required=True)
    c.add_argument("--largest-grid", action="store_true", help="only the launches of the largest grid")
    a = ap.parse_args()
    if a.cmd == "trace":
        trace_summary(a.dir, a.command, a.out)
    else:
        traffic_summary(a.fetch, a.write, a.fetch_copy, a.write_copy, a.kernel, a.command, a.out, a.largest_grid)


if __name__ == "__main__":
    main()
