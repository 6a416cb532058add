"""Summaries of rocprofv3 output for the measurement records under profiles/.

    python -m paper_1905_03344_amd.profiling traffic \\
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --kernel "void k_hsolve_round<4, true>" --source neighbors.hip \\
        --workload square_patch_100^3_1M_fp64 --last 2 --out profiles/X_traffic.json
    python -m paper_1905_03344_amd.profiling stats --csv run_kernel_stats.csv --top 12

`traffic` turns two counter runs (FETCH_SIZE, then WRITE_SIZE, KiB per
dispatch) into HBM bytes per launch of one kernel, each counter scaled by
what it reads for a plain 1 GiB device copy (bench.py --copy-calibration),
and records the SHA-256 of the kernel's source so that a stale record is
ignored.  `stats` prints the kernel-trace summary as a markdown table.
"""
from __future__ import annotations

import argparse
import csv
import hashlib
import json
import os
import statistics
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
COPY_BYTES = 1 << 30


def _rows(path):
    with open(path, newline="") as f:
        return list(csv.DictReader(f))


def per_dispatch(path, name_prefix, counter):
    """Counter values (summed over the per-dispatch records) in dispatch order."""
    vals = {}
    for r in _rows(path):
        if r["Counter_Name"] != counter or not r["Kernel_Name"].startswith(name_prefix):
            continue
        d = int(r["Dispatch_Id"])
        vals[d] = vals.get(d, 0.0) + float(r["Counter_Value"])
    return [vals[d] for d in sorted(vals)]


def source_digest(path):
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def traffic(a):
    fetch = per_dispatch(a.fetch, a.kernel, "FETCH_SIZE")[-a.last:]
    write = per_dispatch(a.write, a.kernel, "WRITE_SIZE")[-a.last:]
    if not fetch or not write:
        raise SystemExit(f"no dispatches of {a.kernel!r}")
    cf = per_dispatch(a.copy_fetch, "__amd_rocclr_copyBuffer", "FETCH_SIZE")
    cw = per_dispatch(a.copy_write, "__amd_rocclr_copyBuffer", "WRITE_SIZE")
    f_scale = COPY_BYTES / (statistics.median(cf) * 1024.0)
    w_scale = COPY_BYTES / (statistics.median(cw) * 1024.0)
    f_kib, w_kib = statistics.median(fetch), statistics.median(write)
    rec = {
        "kernel": a.kernel,
        "workload": a.workload,
        "fetch_kib_per_dispatch": f_kib,
        "write_kib_per_dispatch": w_kib,
        "fetch_scale": round(f_scale, 4),
        "write_scale": round(w_scale, 4),
        "bytes_per_launch": int(f_kib * 1024.0 * f_scale + w_kib * 1024.0 * w_scale),
        "dispatches_used": a.last,
        "source": a.source,
        "source_sha256_16": source_digest(os.path.join(HERE, "csrc", a.source)),
        "commands": a.commands,
    }
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def stats(a):
    rows = _rows(a.csv)
    rows.sort(key=lambda r: -float(r["TotalDurationNs"]))
    total = sum(float(r["TotalDurationNs"]) for r in rows)
    print("| kernel | calls | total ms | avg us | share |")
    print("|---|---|---|---|---|")
    for r in rows[: a.top]:
        t = float(r["TotalDurationNs"])
        print(f"| `{r['Name'][:80]}` | {r['Calls']} | {t / 1e6:.3f} | "
              f"{float(r['AverageNs']) / 1e3:.1f} | {100 * t / total:.1f}% |")


def main(argv=None):
    ap = argparse.ArgumentParser()
    sub = ap.add_subparsers(dest="cmd", required=True)
    t = sub.add_parser("traffic")
    for k in ("fetch", "write", "copy_fetch", "copy_write", "kernel", "source", "workload", "out"):
        t.add_argument("--" + k.replace("_", "-"), required=True)
    t.add_argument("--last", type=int, default=2)
    t.add_argument("--commands", nargs="*", default=[])
    s = sub.add_parser("stats")
    s.add_argument("--csv", required=True)
    s.add_argument("--top", type=int, default=12)
    a = ap.parse_args(argv)
    traffic(a) if a.cmd == "traffic" else stats(a)


if __name__ == "__main__":
    main(sys.argv[1:])
