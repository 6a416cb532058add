"""Summaries of rocprofv3 output for the measurement records under profiles/.

    python -m paper_1905_03344_amd.profiling traffic \\
        --fetch F.csv --write W.csv --copy-fetch CF.csv --copy-write CW.csv \\
        --kernel "void k_hsolve_round<4, true>" --source neighbors.hip \\
        --workload square_patch_100^3_1M_fp64 --last 2 --out profiles/X_traffic.json
    python -m paper_1905_03344_amd.profiling stats --csv run_kernel_stats.csv --top 12
    python -m paper_1905_03344_amd.profiling counters --csv A.csv B.csv \\
        --kernel "void k_hsolve_round<4, true>" --source neighbors.hip \\
        --workload "square_patch_400^3_64M" [--traffic T.json --duration-us D] --out C.json

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


# MI355X: 256 compute units of 4 SIMDs each in 8 XCDs; rocprofv3 reports
# GRBM_GUI_ACTIVE summed over the XCDs (a dispatch reads 8x its duration in
# cycles), so the busy fractions divide by the per-XCD value
CU_NUM = 256
SIMD_NUM = 4 * CU_NUM
XCD_NUM = 8


def counters(a):
    """Busy fractions of one kernel from counter passes (per dispatch, the
    median of the last `last` dispatches; every pass run on the same
    command; g = GRBM_GUI_ACTIVE / XCD_NUM, the kernel's cycles):
      valu_busy = SQ_ACTIVE_INST_VALU * 4 / SIMD_NUM / GRBM_GUI_ACTIVE
      valu_lanes = SQ_THREAD_CYCLES_VALU / (64 SQ_ACTIVE_INST_VALU)
      mfma_busy = SQ_VALU_MFMA_BUSY_CYCLES / (4 CU_NUM GRBM_GUI_ACTIVE)
      ta_busy = TA_TA_BUSY (summed over units) / (CU_NUM GRBM_GUI_ACTIVE)
      lds_busy = SQ_ACTIVE_INST_LDS * 4 / SIMD_NUM / GRBM_GUI_ACTIVE
    and, with --traffic, the measured HBM fraction: the traffic record's
    bytes per launch over the kernel's average duration (--duration-us)
    against 8 TB/s.  `bound` names the busiest of VALU, TA and HBM."""
    vals = {}
    for path in a.csv:
        seen = {}
        for r in _rows(path):
            if not r["Kernel_Name"].startswith(a.kernel):
                continue
            d = int(r["Dispatch_Id"])
            key = (r["Counter_Name"], d)
            seen[key] = seen.get(key, 0.0) + float(r["Counter_Value"])
        names = {k[0] for k in seen}
        for nm in names:
            ds = sorted(d for (c, d) in seen if c == nm)[-a.last:]
            vals[nm] = statistics.median(seen[(nm, d)] for d in ds)
    g = vals.get("GRBM_GUI_ACTIVE")
    g = g / XCD_NUM if g else g
    rec = {"kernel": a.kernel, "workload": a.workload, "raw_per_dispatch": vals}
    if g:
        if "SQ_ACTIVE_INST_VALU" in vals:
            rec["valu_busy"] = round(vals["SQ_ACTIVE_INST_VALU"] * 4 / SIMD_NUM / g, 4)
            if "SQ_THREAD_CYCLES_VALU" in vals and vals["SQ_ACTIVE_INST_VALU"] > 0:
                rec["valu_lanes"] = round(vals["SQ_THREAD_CYCLES_VALU"] /
                                          (64.0 * vals["SQ_ACTIVE_INST_VALU"]), 4)
        if "SQ_VALU_MFMA_BUSY_CYCLES" in vals:
            rec["mfma_busy"] = round(vals["SQ_VALU_MFMA_BUSY_CYCLES"] / (4.0 * CU_NUM * g), 4)
        if "TA_TA_BUSY" in vals:
            rec["ta_busy"] = round(vals["TA_TA_BUSY"] / (CU_NUM * g), 4)
        if "SQ_ACTIVE_INST_LDS" in vals:
            rec["lds_busy"] = round(vals["SQ_ACTIVE_INST_LDS"] * 4 / SIMD_NUM / g, 4)
    if a.traffic and a.duration_us:
        with open(a.traffic) as f:
            t = json.load(f)
        rec["hbm_frac_measured"] = round(t["bytes_per_launch"] / (a.duration_us * 1e-6) / 8e12, 4)
    cand = {k: rec[k] for k in ("valu_busy", "ta_busy", "hbm_frac_measured") if k in rec}
    if cand:
        top = max(cand, key=cand.get)
        rec["bound"] = {"valu_busy": "alu", "ta_busy": "alu", "hbm_frac_measured": "hbm"}[top]
        rec["busiest"] = top
    rec["source"] = a.source
    rec["source_sha256_16"] = source_digest(os.path.join(HERE, "csrc", a.source))
    rec["commands"] = a.commands
    with open(a.out, "w") as f:
        json.dump(rec, f, indent=1)
        f.write("\n")
    print(json.dumps(rec))


def dispatches(a):
    """Average duration of the last `last` dispatches of each kernel whose
    name starts with one of the prefixes, from a rocprofv3 kernel trace (the
    timed steps of a run, after its t = 0 evaluation and warmup steps)."""
    rows = _rows(a.trace)
    if a.anchor:
        # per step: the dispatches between consecutive starts of the anchor
        # kernel (the first kernel of a step), over the last `last` starts
        anc = sorted(int(r["Start_Timestamp"]) for r in rows
                     if r["Kernel_Name"].startswith(a.anchor))[-a.last:]
        nstep = len(anc) - 1
        lo, hi = anc[0], anc[-1]
        inside = [r for r in rows if lo <= int(r["Start_Timestamp"]) < hi]
        print("| kernel | dispatches per step | us per step (%d steps) |" % nstep)
        print("|---|---|---|")
        for pre in a.kernel:
            ds = [r for r in inside if r["Kernel_Name"].startswith(pre)]
            if not ds:
                continue
            us = sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in ds)
            print(f"| `{pre}` | {len(ds) / nstep:g} | {us / nstep:.1f} |")
        tot = sum((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in inside)
        print(f"| all kernels | {len(inside) / nstep:g} | {tot / nstep:.1f} |")
        return
    print("| kernel | dispatches | avg us (last %d) |" % a.last)
    print("|---|---|---|")
    for pre in a.kernel:
        ds = [r for r in rows if r["Kernel_Name"].startswith(pre)]
        ds.sort(key=lambda r: int(r["Start_Timestamp"]))
        tail = ds[-a.last:]
        if not tail:
            continue
        us = [(int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3 for r in tail]
        print(f"| `{pre}` | {len(ds)} | {sum(us) / len(us):.1f} |")


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
    d = sub.add_parser("dispatches")
    d.add_argument("--trace", required=True)
    d.add_argument("--kernel", nargs="+", required=True)
    d.add_argument("--last", type=int, default=3)
    d.add_argument("--anchor", default=None,
                   help="first kernel of a step: report per-step sums between its last "
                        "`--last` starts")
    c = sub.add_parser("counters")
    c.add_argument("--csv", nargs="+", required=True)
    for k in ("kernel", "source", "workload", "out"):
        c.add_argument("--" + k, required=True)
    c.add_argument("--traffic")
    c.add_argument("--duration-us", type=float)
    c.add_argument("--last", type=int, default=1)
    c.add_argument("--commands", nargs="*", default=[])
    a = ap.parse_args(argv)
    {"traffic": traffic, "stats": stats, "counters": counters, "dispatches": dispatches}[a.cmd](a)


if __name__ == "__main__":
    main(sys.argv[1:])
