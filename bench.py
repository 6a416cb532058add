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
# per candidate tested by the h iteration's counting walk: 3 differences,
# 3 squares, 2 adds (the two comparisons against the shell bounds not counted)
HSOLVE_FLOPS_PER_CANDIDATE = 8
# per gather-set pair of the density kernel: differences 3, r^2 5, the
# complement test 3, sqrt 1, W 8, sum 2, dW/dr 7, /r 1, v_ij 3, dot 5, sum 2
DENSITY_FLOPS_PER_PAIR = 40
# algorithmic HBM bytes of the density kernel: own x y z v(3) m h (64 B),
# nc (4 B), writes rho divv (16 B) and the E row count (4 B), plus 4 B per
# list entry read
DENSITY_BYTES_PER_PARTICLE = 88
# of the first counting walk: own x y z h key (36 B) read, h nc flags state
# (about 24 B) written, 4 B per gather-set entry written
HWALK_BYTES_PER_PARTICLE = 60
FP64_PEAK_TFLOPS = 78.6
HBM_PEAK_GBS = 8000.0
# algorithmic HBM bytes of the force kernel per particle, besides 4 B per list
# entry: own fields x y z v(3) m h rho P c (88 B), nc and E count (8 B), and
# the writes a(3) du (32 B); neighbour data are re-reads of those fields
FORCE_BYTES_PER_PARTICLE = 128
FORCE_BYTES_PER_ENTRY = 4
CSRC = os.path.join(ROOT, "paper_1905_03344_amd", "csrc")
# kernel -> (stage timed around its launch alone, source file holding it)
KERNELS = {"k_hsolve_round": ("hwalk", "neighbors.hip"),
           "k_forces": ("forces", "physics.hip"),
           "k_density": ("density", "physics.hip")}

CONFIG_NAMES = {
    1: "square_patch_20^3_8k_fp64",
    2: "square_patch_100^3_1M_fp64",
    3: "square_patch_200^3_8M",
    4: "clumpy_1M",
    5: "square_patch_400^3_64M",
}


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def cpu_baseline(config: int, kernel: int = 0, integrator: int = 0, grad_h: bool = False,
                 gradients: int = 0):
    """The oracle (as it stands) timed on this host for one kick-drift-kick
    step of the benchmark workload itself (the t = 0 evaluation that precedes
    it is not timed)."""
    import oracle as O
    from paper_1905_03344_amd import inputs
    ic = inputs.config_ic(config)
    st = O.State(ic, O.Params(kernel=kernel, integrator=integrator, grad_h=grad_h,
                              gradients=gradients))
    st.evaluate(method=1)
    steps = 4 if ic.n <= 2_000_000 else 1
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(None, method=1)
    dt = time.perf_counter() - t0
    return {"value": ic.n * steps / dt, "unit": "particle-updates/s", "cores": O.num_threads(),
            "kind": "oracle",
            "sample": f"{steps} KDK steps (Courant dt) of the full {ic.n}-particle workload "
                      f"after an untimed t=0 evaluation, {dt:.2f} s"}


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def measured_traffic(kernel, workload):
    """HBM bytes per launch of `kernel` on `workload` from the committed PMC
    summary (profiles/<kernel>_<workload>_traffic.json), or None when there
    is none or the kernel's source changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_traffic.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    src = os.path.join(CSRC, KERNELS[kernel][1])
    if t.get("source_sha256_16") != source_digest(src):
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
    ap.add_argument("--integrator", default="kdk", choices=["kdk", "ab2"],
                    help="kick-drift-kick, or its positions with Adams-Bashforth energy")
    ap.add_argument("--gradients", default="kernel", choices=["kernel", "iad"],
                    help="gradient estimator of the momentum and energy sums (iad: plain form)")
    ap.add_argument("--walk-defer-group", type=int, default=None,
                    help="first-round walk sub-groups up to this size go to the per-particle "
                         "tail (default: 16 on the clumpy mixture, else the library's 4)")
    ap.add_argument("--grad-h", action="store_true",
                    help="grad-h correction terms in the momentum and energy sums (plain form)")
    ap.add_argument("--kernel", default="m4", choices=["m4", "wendland", "sinc5"],
                    help="smoothing kernel of the density and force sums")
    ap.add_argument("--walk-prefilter", default="matrix", choices=["matrix", "none"],
                    help="candidate test of the h-iteration walk: bf16 Gram prefilter on the "
                         "matrix cores with an exact FP64 band, or FP64 for every candidate")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}); the multi-GPU "
              "decomposition is designed but not implemented", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1905_03344_amd import ffi, inputs
    from paper_1905_03344_amd.state import Simulation

    torch.cuda.init()
    log(f"bench: config {args.config}, form {args.form}, building inputs")
    learned = args.form == "learned"
    # complement rows: the clumpy mixture's density contrast needs more slots
    extra_slots = 96 if args.config == 4 else 48
    defer = args.walk_defer_group
    if defer is None:
        defer = 16 if args.config == 4 else 0
    # the learned form is timed on seed B of the workload after training on
    # 20 plain steps of seed A (the same distribution)
    ic = inputs.config_ic(args.config, seed_offset=100 if learned else 0)
    n = ic.n
    precision = ffi.SPH_FP64 if args.form == "plain" else ffi.SPH_MIXED
    prefilter = (ffi.SPH_PREFILTER_MATRIX if args.walk_prefilter == "matrix"
                 else ffi.SPH_PREFILTER_NONE)
    kernel = {"m4": ffi.SPH_KERNEL_M4, "wendland": ffi.SPH_KERNEL_WENDLAND,
              "sinc5": ffi.SPH_KERNEL_SINC5}[args.kernel]
    integrator = (ffi.SPH_INTEGRATOR_AB2 if args.integrator == "ab2" else ffi.SPH_INTEGRATOR_KDK)
    gradients = (ffi.SPH_GRADIENTS_IAD if args.gradients == "iad" else ffi.SPH_GRADIENTS_KERNEL)
    extra = {}
    if learned:
        from paper_1905_03344_amd import learned as L
        ic_a = inputs.config_ic(args.config)
        tr = Simulation(ic_a, search_div=args.search_div, precision=precision,
                        extra_per_particle=extra_slots, walk_prefilter=prefilter, kernel=kernel,
                        integrator=integrator, grad_h=args.grad_h, gradients=gradients,
                        walk_defer_group=defer)
        tr.evaluate()
        tr.sync()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        # the clumpy mixture's count grows smoothly with h: train towards the
        # band centre; the square patch is a jittered lattice whose count
        # grows in whole shells: train towards the solved h
        mode = ffi.SPH_TARGET_CENTRED if args.config == 4 else ffi.SPH_TARGET_SOLVED
        # 20 harvested plain steps; at 64M rows of 2 steps (128M rows, 4.6 GB)
        harvest_steps = 20 if n <= 8_000_000 else 2
        feat, target = L.harvest(tr, steps=harvest_steps, target_mode=mode)
        tr.sync()
        t1 = time.perf_counter()
        w, norm, losses = L.train(tr, feat, target, seed=inputs.CONFIG_SEEDS[args.config])
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        extra["training"] = {"harvest_steps": harvest_steps, "rows": int(feat.shape[0]),
                             "target": "centred" if mode == ffi.SPH_TARGET_CENTRED else "solved",
                             "harvest_s": round(t1 - t0, 3), "train_s": round(t2 - t1, 3),
                             "epochs": 4, "batch": 8192,
                             "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                             "target_mse_zero_model": float((target.double() ** 2).mean())}
        del feat, target, tr
        torch.cuda.empty_cache()
    sim = Simulation(ic, search_div=args.search_div, precision=precision,
                     h_mode=ffi.SPH_H_LEARNED if learned else ffi.SPH_H_PLAIN,
                     extra_per_particle=extra_slots, walk_prefilter=prefilter, kernel=kernel,
                     integrator=integrator, grad_h=args.grad_h, gradients=gradients,
                     walk_defer_group=defer)
    if learned:
        sim.set_mlp(w, norm)
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

    # work per step: pairs in S (the last step's gather sets plus the mean
    # complement size) and candidates of the h iteration's first walk
    nc = sim.field("nc")
    pairs_l = int(nc.sum().item())
    pairs_e = int(st.extra_total / max(1, args.steps))
    pairs = pairs_l + pairs_e
    cand_first = st.candidates_first / args.steps
    stage_ms = {k: v[0] / max(1, args.steps) for k, v in stages.items()}
    work = {
        "k_hsolve_round": (HSOLVE_FLOPS_PER_CANDIDATE * cand_first,
                           HWALK_BYTES_PER_PARTICLE * n + 4 * pairs_l),
        "k_forces": (FORCE_FLOPS_PER_PAIR * pairs,
                     FORCE_BYTES_PER_PARTICLE * n + FORCE_BYTES_PER_ENTRY * pairs),
        "k_density": (DENSITY_FLOPS_PER_PAIR * pairs_l, DENSITY_BYTES_PER_PARTICLE * n + 4 * pairs_l),
    }
    workload = CONFIG_NAMES[args.config] + ("_seedB" if learned else "")
    kernels = {}
    for kname, (flops, nbytes) in work.items():
        t = stage_ms[KERNELS[kname][0]] * 1e-3
        tf = flops / t / 1e12 if t else 0.0
        gbs = nbytes / t / 1e9 if t else 0.0
        kernels[kname] = {"launch_ms": round(t * 1e3, 4), "flops_per_launch": int(flops),
                          "achieved_tflops": round(tf, 3),
                          "frac_fp64": round(tf / FP64_PEAK_TFLOPS, 4),
                          "algorithmic_bytes": int(nbytes), "achieved_gbs": round(gbs, 1),
                          "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    # the dominant kernel: the longest launch of the step (mixed-form
    # kernels are timed in the same stages; their FP32 work is still
    # priced against the FP64 peak here, a conservative fraction)
    dom = max(kernels, key=lambda k: kernels[k]["launch_ms"])
    kd = kernels[dom]
    roofline = {"bound": "alu", "kernel": dom, "achieved": kd["achieved_tflops"],
                "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s", "frac": kd["frac_fp64"],
                "traffic": measured_traffic(dom, CONFIG_NAMES[args.config]) if args.form == "plain"
                else None,
                "flops_per_launch": kd["flops_per_launch"], "launch_ms": kd["launch_ms"],
                "hbm": {"algorithmic_bytes": kd["algorithmic_bytes"],
                        "achieved": kd["achieved_gbs"], "peak": HBM_PEAK_GBS, "unit": "GB/s",
                        "frac": kd["frac_hbm"]}}
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
        "config": {"workload": workload, "n": n, "form": args.form, "dt": "courant cfl 0.3",
                   "walk_prefilter": args.walk_prefilter, "walk_defer_group": defer or 4,
                   "kernel": args.kernel,
                   "integrator": args.integrator, "grad_h": bool(args.grad_h),
                   "gradients": args.gradients},
        "roofline": roofline,
        "kernels": kernels,
        "stages_ms_per_step": {k: round(v, 4) for k, v in stage_ms.items()},
        "work_per_step": {"pairs_S": pairs, "pairs_L": pairs_l, "pairs_E": pairs_e,
                          "hsolve_candidates_first_walk": cand_first,
                          "hsolve_candidates_all": st.candidates / args.steps,
                          "hsolve_counts_per_particle": st.h_counts / args.steps / n},
        "status": code,
    }
    if learned:
        dec = st.learned_accepted + st.learned_fallback
        extra["accept_rate"] = st.learned_accepted / dec if dec else None
        extra["fallback_rate"] = st.learned_fallback / dec if dec else None
        out["learned"] = extra
    if not args.no_cpu_baseline:
        log("bench: cpu baseline (oracle)")
        out["cpu_baseline"] = cpu_baseline(args.config, kernel, integrator, args.grad_h,
                                           gradients)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
