"""Throughput of full SPH time steps on one MI355X, in particle-updates/s.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 2]
                    [--form plain|mixed|learned] [--no-cpu-baseline]

A step is one kick-drift-kick step of the whole hot path (cell keys, sort,
cell table, smoothing-length iteration with the gather sets, complement
lists, density, EOS, momentum/energy/viscosity with the Courant step, both
kicks).  The default workload is the 100^3 = 1,000,000-particle rotating
square patch in plain FP64 at Courant-limited dt (CFL 0.3).  Inputs are
resident in HBM before the timed region; the t = 0 force evaluation and
the warmup steps are outside it.  Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

# FP64 arithmetic per interaction pair in the force kernel (counted from the
# source: differences 3, r^2 5, sqrt 1, 1/r 1, v_ij 3, v.x 5, two kernel
# gradients 19, average 2, viscosity 10 (19 on the approaching half),
# P/rho^2 2, sums 2, factor 2, acceleration 6, energy 6)
FORCE_FLOPS_PER_PAIR = 67
# per candidate of the h iteration: 3 differences, 3 squares, 2 adds, compare
HSOLVE_FLOPS_PER_CANDIDATE = 9
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes of the force kernel per particle, besides 4 B per list
# entry: own fields x y z v(3) m h rho P c (88 B), nc and E count (8 B), and
# the writes a(3) du (32 B); neighbour data are re-reads of those fields
FORCE_BYTES_PER_PARTICLE = 128
FORCE_BYTES_PER_ENTRY = 4
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "k_forces_traffic.json")
FORCE_SOURCE = os.path.join(ROOT, "paper_1905_03344_amd", "csrc", "physics.hip")

CONFIG_NAMES = {
    1: "square_patch_20^3_8k_fp64",
    2: "square_patch_100^3_1M_fp64",
    3: "square_patch_200^3_8M",
    4: "clumpy_1M",
    5: "square_patch_400^3_64M",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(config: int):
    """The oracle (as it stands) timed on this host for one kick-drift-kick
    step of the benchmark workload itself (the t = 0 evaluation that precedes
    it is not timed)."""
    import oracle as O
    from paper_1905_03344_amd import inputs
    ic = inputs.config_ic(config)
    st = O.State(ic)
    st.evaluate(method=1)
    t0 = time.perf_counter()
    st.step(None, method=1)
    dt = time.perf_counter() - t0
    return {"value": ic.n / dt, "unit": "particle-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"one KDK step (Courant dt) of the full {ic.n}-particle workload "
                      f"after an untimed t=0 evaluation, {dt:.2f} s"}


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic():
    """HBM bytes per k_forces launch from the committed PMC summary, or None
    when the kernel source changed since the counters were taken."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("source_sha256_16") != source_digest(FORCE_SOURCE):
        return None
    return t.get("bytes_per_launch")


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=2)
    ap.add_argument("--form", default="plain", choices=["plain", "mixed", "learned"])
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--search-div", type=int, default=2)
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is a design, not part of this build", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1905_03344_amd import ffi, inputs
    from paper_1905_03344_amd.state import Simulation

    torch.cuda.init()
    log(f"bench: config {args.config}, form {args.form}, building inputs")
    ic = inputs.config_ic(args.config)
    n = ic.n
    precision = ffi.SPH_FP64 if args.form == "plain" else ffi.SPH_MIXED
    sim = Simulation(ic, search_div=args.search_div, precision=precision)
    log(f"bench: n={n} max_level={sim.params.max_level} workspace={sim.ws_bytes/2**20:.1f} MiB")
    sim.evaluate()
    sim.sync()
    for _ in range(args.warmup):
        sim.step(0.0)
    sim.sync()
    log("bench: warmup done")
    stream = sim.stream
    ffi.sph_timing(sim.ctx, True)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        sim.step(0.0)
    e1.record(stream)
    torch.cuda.synchronize()
    total_ms = e0.elapsed_time(e1)
    stages = ffi.sph_timing_read(sim.ctx)
    ffi.sph_timing(sim.ctx, False)
    code, st = sim.sync()
    ms_per_step = total_ms / args.steps
    value = n * args.steps / (total_ms * 1e-3)

    # work of the last step: pairs in S and candidates of the h iteration
    nc = sim.field("nc")
    pairs_l = int(nc.sum().item())
    pairs_e = int(st.extra_total / max(1, args.steps))
    pairs = pairs_l + pairs_e
    cand_per_step = st.candidates / args.steps
    stage_ms = {k: v[0] / max(1, args.steps) for k, v in stages.items()}
    force_flops = FORCE_FLOPS_PER_PAIR * pairs
    hs_flops = HSOLVE_FLOPS_PER_CANDIDATE * cand_per_step
    t_force = stage_ms["forces"] * 1e-3
    force_tf = force_flops / t_force / 1e12 if t_force else 0
    hs_tf = hs_flops / (stage_ms["hsolve"] * 1e-3) / 1e12 if stage_ms["hsolve"] else 0
    force_bytes = FORCE_BYTES_PER_PARTICLE * n + FORCE_BYTES_PER_ENTRY * pairs
    force_gbs = force_bytes / t_force / 1e9 if t_force else 0
    traffic = measured_traffic()
    # the dominant kernel: k_forces has the longest single launch of the step
    roofline = {"bound": "alu", "kernel": "k_forces", "achieved": round(force_tf, 3),
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                "frac": round(force_tf / FP64_PEAK_TFLOPS, 4), "traffic": traffic,
                "flops_per_launch": force_flops, "launch_ms": round(stage_ms["forces"], 4),
                "hbm": {"algorithmic_bytes": force_bytes, "achieved": round(force_gbs, 1),
                        "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": round(force_gbs / HBM_PEAK_GBS, 4)}}
    out = {
        "metric": "particle-updates/s per full SPH step",
        "value": value,
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_per_step,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if args.form == "plain" else "f32/f64",
        "data": "synthetic",
        "config": {"workload": CONFIG_NAMES[args.config], "n": n, "form": args.form,
                   "dt": "courant cfl 0.3"},
        "roofline": roofline,
        "stages_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "work_per_step": {"pairs_S": pairs, "pairs_L": pairs_l, "pairs_E": pairs_e,
                          "hsolve_candidates": cand_per_step,
                          "hsolve_counts_per_particle": st.h_counts / args.steps / n,
                          "force_tflops": round(force_tf, 3), "hsolve_tflops": round(hs_tf, 3)},
        "status": code,
    }
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.config)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
