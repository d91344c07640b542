"""Summaries of rocprofv3 CSV output (kernel-trace stats, FETCH_SIZE and
WRITE_SIZE counter passes) as short markdown, plus the per-launch HBM traffic
of the neighbour-search phase that the benchmark reports.

    python -m paper_2607_05504_amd.profsum stats  <run_kernel_stats.csv>
    python -m paper_2607_05504_amd.profsum traffic <fetch_dir> <write_dir> \
        <copy_fetch_dir> <copy_write_dir> <copy_mib> <workload> [traffic.json]

The counters are scaled by what the same counters read for a plain copy of
known size (copy_mib MiB read and written): factor = known KiB / counted KiB.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import re
import sys


def short(name: str) -> str:
    n = re.sub(r"\(anonymous namespace\)::", "", name)
    n = n.replace("void ", "")
    m = re.match(r"([^(]*)", n)
    return (m.group(1) if m else n).strip()


def stats(path: str) -> str:
    rows = list(csv.DictReader(open(path)))
    out = ["| kernel | calls | avg us | total us | % |", "|---|---:|---:|---:|---:|"]
    for r in sorted(rows, key=lambda r: -float(r["TotalDurationNs"])):
        out.append(f"| {short(r['Name'])[:60]} | {r['Calls']} | {float(r['AverageNs']) / 1e3:.2f} "
                   f"| {float(r['TotalDurationNs']) / 1e3:.1f} | {float(r['Percentage']):.2f} |")
    return "\n".join(out)


def counters(d: str) -> dict:
    agg = collections.defaultdict(list)
    for r in csv.DictReader(open(os.path.join(d, "run_counter_collection.csv"))):
        agg[short(r["Kernel_Name"])].append(float(r["Counter_Value"]))
    return agg


def copy_factor(d: str, mib: int) -> float:
    vals = counters(d)["__amd_rocclr_copyBuffer"]
    big = [v for v in vals if v > mib * 1024 * 0.25]     # the copies of the probe itself
    return (mib * 1024.0) / (sum(big) / len(big))


KNN_KERNELS = ("k_knn_list", "k_knn_bucket", "k_knn_team")
KNN_SOURCES = tuple(os.path.join(os.path.dirname(os.path.abspath(__file__)), "csrc", f)
                    for f in ("knn.hip", "sidm_internal.h"))


def source_hash(paths=KNN_SOURCES) -> str:
    """Identifies the kernel sources the counters were taken on (the search
    and the shared header with its launch mapping); a traffic figure taken on
    other sources is stale."""
    h = hashlib.sha256()
    for p in paths:
        h.update(open(p, "rb").read())
    return h.hexdigest()[:16]


def traffic(fd, wd, cfd, cwd, mib, workload, out_json=None) -> str:
    ff, wf = copy_factor(cfd, mib), copy_factor(cwd, mib)
    fetch, write = counters(fd), counters(wd)
    lines = [f"copy calibration ({mib} MiB read + written): FETCH_SIZE x {ff:.3f}, "
             f"WRITE_SIZE x {wf:.3f}", "",
             "| kernel | dispatches | FETCH KiB/dispatch | WRITE KiB/dispatch | HBM MB/dispatch (scaled) |",
             "|---|---:|---:|---:|---:|"]
    names = sorted(set(fetch) | set(write),
                   key=lambda n: -(sum(fetch.get(n, [0])) / max(1, len(fetch.get(n, [1])))))
    knn_total = 0.0
    for n in names:
        f = fetch.get(n, [0.0])
        w = write.get(n, [0.0])
        fa, wa = sum(f) / len(f), sum(w) / len(w)
        mb = (fa * ff + wa * wf) * 1024 / 1e6
        lines.append(f"| {n[:60]} | {len(f)} | {fa:.1f} | {wa:.1f} | {mb:.3f} |")
        if n.split("<")[0] in KNN_KERNELS:
            knn_total += (fa * ff + wa * wf) * 1024 * len(f)
    # one neighbour search per scatter step; a search over more targets than
    # one batch holds is several dispatches of each kernel
    calls = len(fetch.get("k_step_reset", [])) or 1
    knn_bytes = knn_total / calls
    lines.append("")
    lines.append(f"neighbour-search phase HBM traffic per launch ({calls} launches, "
                 f"all batches of one launch summed): {knn_bytes / 1e6:.3f} MB")
    if out_json:
        tr = json.load(open(out_json)) if os.path.exists(out_json) else {}
        tr.setdefault(workload, {})["knn"] = {"bytes_per_launch": knn_bytes,
                                              "fetch_factor": ff, "write_factor": wf,
                                              "source": source_hash()}
        with open(out_json, "w") as fh:
            json.dump(tr, fh, indent=1)
    return "\n".join(lines)


if __name__ == "__main__":
    if sys.argv[1] == "stats":
        print(stats(sys.argv[2]))
    elif sys.argv[1] == "traffic":
        a = sys.argv[2:]
        print(traffic(a[0], a[1], a[2], a[3], int(a[4]), a[5], a[6] if len(a) > 6 else None))
    else:
        raise SystemExit(__doc__)
