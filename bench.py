"""Throughput of full SPH time steps on one MI355X, in particle-updates/s.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--config 5]
                    [--form headline|plain|mixed|learned] [--no-cpu-baseline]

A step is one kick-drift-kick step of the whole hot path (cell keys, sort,
cell table, smoothing-length iteration with the gather sets, complement
lists, density, EOS, momentum/energy/viscosity with the Courant step, both
kicks).  The default workload is the largest single-GPU configuration, the
400^3 = 64,000,000-particle rotating square patch at Courant-limited dt
(CFL 0.3), and the default form `headline` times both production forms on
the same input, one after the other (each freed before the next):

  * plain FP64 -- `value`, `ms_per_step` and `roofline` are this form's;
  * FP32-mixed pair arithmetic with the learned smoothing length and plain
    fallback, its MLP trained on the device on plain steps of another seed
    of the same distribution (training time reported, not timed) --
    reported under `forms` with its speedup over plain FP64 and its
    fallback rate.

Each form also reports the conservation drift over its timed steps, and,
from the cpu_baseline leg (the only part of this script that runs the CPU
oracle), its error against the oracle on a cube of particles cut from its
final state (`accuracy`).  Inputs are resident in HBM before the timed
region; the t = 0 force evaluation and the warmup steps are outside it.
Prints one JSON line.
"""
from __future__ import annotations

import argparse
import json
import os
import platform
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
# the counting pass of the h iteration, priced by its algorithmic work, not
# by what the implementation tests: the 27 cells of c/2h ~ 1.04 around a
# particle of the jittered lattice hold ~824 candidates, each a 3-difference,
# 3-square, 2-add r^2 (8 FP64 flops; the comparisons are not counted)
HSOLVE_CANDIDATES_PER_PARTICLE = 824
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
    1: "square_patch_20^3_8k",
    2: "square_patch_100^3_1M",
    3: "square_patch_200^3_8M",
    4: "clumpy_1M",
    5: "square_patch_400^3_64M",
}
# half-width of the cube cut from the final state for the accuracy check
# (square patches; the clumpy mixture uses a cube around its densest clump)
CUBE_HALF = {1: 0.2, 2: 0.1, 3: 0.08, 5: 0.06}
TOL_FP64 = 1e-12
TOL_MIXED = 1e-5


def log(msg):
    print(msg, file=sys.stderr, flush=True)


def host_info():
    model = platform.processor() or ""
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    model = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    return {"cpu_model": model, "nproc": os.cpu_count()}


def source_digest(path):
    import hashlib
    with open(path, "rb") as f:
        return hashlib.sha256(f.read()).hexdigest()[:16]


def profile_record(kernel, workload, kind):
    """A committed PMC summary (profiles/<kernel>_<workload>_<kind>.json), or
    None when there is none or the kernel's source changed since the counters
    were taken."""
    path = os.path.join(ROOT, "profiles", f"{kernel}_{workload}_{kind}.json")
    try:
        with open(path) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    src = os.path.join(CSRC, KERNELS[kernel][1])
    if t.get("source_sha256_16") != source_digest(src):
        return None
    return t


def copy_calibration(nbytes=1 << 30, reps=3):
    """A plain device copy of known size, for scaling FETCH_SIZE/WRITE_SIZE."""
    import torch
    a = torch.empty(nbytes // 8, dtype=torch.float64, device="cuda").fill_(1.0)
    b = torch.empty_like(a)
    for _ in range(reps):
        b.copy_(a)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes": nbytes, "reps": reps}), flush=True)


# ---------------------------------------------------------------------------
# one timed form
# ---------------------------------------------------------------------------
def _conservation_scales(sim):
    """sum m |v| and sum m |x| |v| of the current state (device reductions;
    the scales the momentum and angular-momentum drifts are reported in)."""
    import torch
    m = sim.field("m")
    v = torch.sqrt(sim.field("vx") ** 2 + sim.field("vy") ** 2 + sim.field("vz") ** 2)
    r = torch.sqrt(sim.field("x") ** 2 + sim.field("y") ** 2 + sim.field("z") ** 2)
    return float((m * v).sum()), float((m * r * v).sum())


def _drift(c0, c1, pscale, lscale):
    import numpy as np
    return {"energy_rel": float((c1[6] - c0[6]) / abs(c0[6])),
            "momentum_over_sum_m_abs_v": float(np.linalg.norm(c1[:3] - c0[:3]) / pscale),
            "angular_momentum_over_sum_m_abs_x_abs_v":
                float(np.linalg.norm(c1[3:6] - c0[3:6]) / lscale)}


def _cube_sample(sim, config, half):
    """Fields of the particles in a cube of the current state (selected on
    the device), with the velocity and energy the last force evaluation
    used: what the accuracy check needs to re-evaluate them on the CPU."""
    import numpy as np
    import torch
    x, y, z = sim.field("x"), sim.field("y"), sim.field("z")
    if config == 4:
        # about the densest clump (the particle with the smallest h), kept
        # inside [0.1, 0.9]^3 where the background bounds h (outside the unit
        # cube only sparse clump tails remain, with h up to ~1)
        k = int(torch.argmin(sim.field("h")))
        c = tuple(min(max(float(a[k]), 0.25), 0.75) for a in (x, y, z))
    else:
        c = (0.0, 0.0, 0.0)
    sel = ((x - c[0]).abs() < half) & ((y - c[1]).abs() < half) & ((z - c[2]).abs() < half)
    names = {"x": "x", "y": "y", "z": "z", "vx": "pvx", "vy": "pvy", "vz": "pvz", "m": "m",
             "h": "h", "u": "pu", "rho": "rho", "divv": "divv", "ax": "ax", "ay": "ay",
             "az": "az", "du": "du", "nc": "nc", "p": "p", "c": "c"}
    f = {k: sim.field(v)[sel].cpu().numpy() for k, v in names.items()}
    f["centre"] = np.array(c)
    f["half"] = half
    return f


def run_form(args, config, form, ic, precision_mixed, learned_weights=None, defer=0,
             extra_slots=48, want_sample=True):
    """Time `args.steps` KDK steps of one form on ic after an untimed t = 0
    evaluation and `args.warmup` steps.  Returns a record and the cube
    sample (or None)."""
    import torch
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation

    learned = learned_weights is not None
    sim = Simulation(ic, search_div=args.search_div, max_level=args.max_level,
                     precision=ffi.SPH_MIXED if precision_mixed else ffi.SPH_FP64,
                     h_mode=ffi.SPH_H_LEARNED if learned else ffi.SPH_H_PLAIN,
                     extra_per_particle=extra_slots, walk_prefilter=args.prefilter,
                     kernel=args.kernel_id, integrator=args.integrator_id, grad_h=args.grad_h,
                     gradients=args.gradients_id, walk_defer_group=defer,
                     walk_strategy=args.strategy_id, learned_try_shell=args.try_shell_id)
    if learned:
        sim.set_mlp(*learned_weights)
    n = sim.n
    log(f"bench: {form}: n={n} max_level={sim.params.max_level} "
        f"workspace={sim.ws_bytes / 2**30:.2f} GiB")
    sim.evaluate()
    sim.sync()
    for _ in range(args.warmup):
        sim.step(0.0)
    sim.sync()
    c0 = sim.conservation()
    pscale, lscale = _conservation_scales(sim)
    log(f"bench: {form}: warmup done")
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
    c1 = sim.conservation()
    ms = total_ms / args.steps
    nc = sim.field("nc")
    pairs_l = int(nc.sum().item())
    pairs_e = int(st.extra_total / max(1, args.steps))
    rec = {
        "form": form, "n": n, "ms_per_step": ms, "value": n * args.steps / (total_ms * 1e-3),
        "stages_ms_per_step": {k: round(v[0] / max(1, args.steps), 4) for k, v in stages.items()},
        "work_per_step": {"pairs_S": pairs_l + pairs_e, "pairs_L": pairs_l, "pairs_E": pairs_e,
                          "hsolve_candidates_first_walk": st.candidates_first / args.steps,
                          "hsolve_candidates_all": st.candidates / args.steps,
                          "hsolve_counts_per_particle": st.h_counts / args.steps / n},
        "drift_over_timed_steps": _drift(c0, c1, pscale, lscale),
        "status": code,
    }
    if learned:
        dec = st.learned_accepted + st.learned_fallback
        rec["accept_rate"] = st.learned_accepted / dec if dec else None
        rec["fallback_rate"] = st.learned_fallback / dec if dec else None
    sample = None
    if want_sample and (config in CUBE_HALF or config == 4):
        sample = _cube_sample(sim, config, CUBE_HALF.get(config, 0.15))
        sample["mixed"] = bool(precision_mixed)
    del sim
    torch.cuda.empty_cache()
    return rec, sample


def train_learned(args, config, ic_train, defer, extra_slots):
    """Harvest plain steps of the training input, fit the MLP on the device.
    Returns ((weights, norm12), training record)."""
    import torch
    from paper_1905_03344_amd import ffi, inputs
    from paper_1905_03344_amd import learned as L
    from paper_1905_03344_amd.state import Simulation

    tr = Simulation(ic_train, search_div=args.search_div, max_level=args.max_level,
                    precision=ffi.SPH_MIXED,
                    extra_per_particle=extra_slots, walk_prefilter=args.prefilter,
                    kernel=args.kernel_id, integrator=args.integrator_id, grad_h=args.grad_h,
                    gradients=args.gradients_id, walk_defer_group=defer,
                    walk_strategy=args.strategy_id)
    tr.evaluate()
    tr.sync()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    # the clumpy mixture's count grows smoothly with h: train towards the
    # band centre; the square patch is a jittered lattice whose count grows
    # in whole shells: train towards the solved h
    mode = ffi.SPH_TARGET_CENTRED if config == 4 else ffi.SPH_TARGET_SOLVED
    n = tr.n
    # 20 harvested plain steps; above 8M particles rows of 4 steps after 2
    # unharvested ones (the timed steps come after 2 warmup steps), 2 epochs
    big = n > 8_000_000
    skip, harvest_steps, epochs = (2, 4, 2) if big else (0, 20, 4)
    for _ in range(skip):
        tr.step(0.0)
    feat, target = L.harvest(tr, steps=harvest_steps, target_mode=mode)
    tr.sync()
    t1 = time.perf_counter()
    w, norm, losses = L.train(tr, feat, target, seed=inputs.CONFIG_SEEDS[config], epochs=epochs)
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    rec = {"steps_before_harvest": skip, "harvest_steps": harvest_steps,
           "rows": int(feat.shape[0]),
           "target": "centred" if mode == ffi.SPH_TARGET_CENTRED else "solved",
           "harvest_s": round(t1 - t0, 3), "train_s": round(t2 - t1, 3),
           "epochs": epochs, "batch": 8192,
           "loss_first": float(losses[0]), "loss_last": float(losses[-1]),
           "target_mse_zero_model": float((target.double() ** 2).mean())}
    del feat, target, tr
    torch.cuda.empty_cache()
    return (w, norm), rec


# ---------------------------------------------------------------------------
# the CPU oracle: accuracy of the GPU forms and the oracle's own throughput
# ---------------------------------------------------------------------------
def _accuracy(O, f, params_kw):
    """Re-evaluate a cube sample on the CPU oracle at the GPU's own h (gather
    counts, interaction sets, density, EOS, forces) and compare the particles
    at least 4 h_max inside the cube: their sums involve only particles
    within 4 h of them, all of which the cube holds."""
    import numpy as np
    hmax = float(f["h"].max())
    c, half = f["centre"], float(f["half"])
    lo = tuple(float(v) for v in c - half)
    hi = tuple(float(v) for v in c + half)
    per = (0, 0, 0)
    t0 = time.perf_counter()
    nc = O.count(f["x"], f["y"], f["z"], f["h"], per, lo, hi, 1)
    off, idx = O.lists(f["x"], f["y"], f["z"], f["h"], per, lo, hi, 1)
    kern = params_kw["kernel"]
    rho, divv, dvmag, omega = O.density(f["x"], f["y"], f["z"], f["vx"], f["vy"], f["vz"],
                                        f["m"], f["h"], per, lo, hi, off, idx, with_mag=True,
                                        kernel=kern, with_omega=True)
    P, cs = O.eos(rho, f["u"])
    iad = None
    if params_kw["iad"]:
        iad, _ = O.iad_matrices(f["x"], f["y"], f["z"], f["m"], rho, f["h"], per, lo, hi, off,
                                idx, kernel=kern)
    ax, ay, az, du, dt_i, amag, dumag = O.forces(f["x"], f["y"], f["z"], f["vx"], f["vy"],
                                                 f["vz"], f["m"], f["h"], rho, P, cs, per, lo, hi,
                                                 off, idx, 1.0, 2.0, 0.01, 0.3, with_mag=True,
                                                 kernel=kern,
                                                 omega=omega if params_kw["grad_h"] else None,
                                                 iad=iad)
    t_oracle = time.perf_counter() - t0
    inner = half - 4.0 * hmax * 1.01
    d = np.maximum.reduce([np.abs(f["x"] - c[0]), np.abs(f["y"] - c[1]), np.abs(f["z"] - c[2])])
    deep = d < inner
    if not deep.any():
        return {"sample": f"{len(f['x'])}-particle cube of half-width {half}: none is "
                          f"4 h_max = {4 * hmax:.3g} inside it", "compared": 0}
    a_gpu = np.stack([f["ax"], f["ay"], f["az"]], 1)[deep]
    a_ref = np.stack([ax, ay, az], 1)[deep]
    da = np.linalg.norm(a_gpu - a_ref, axis=1)
    tol = TOL_MIXED if f["mixed"] else TOL_FP64
    out = {
        "sample": f"{len(f['x'])}-particle cube of half-width {half} about "
                  f"({c[0]:.4g}, {c[1]:.4g}, {c[2]:.4g}) cut from the final state; "
                  f"{int(deep.sum())} particles 4 h_max inside it compared",
        "compared": int(deep.sum()),
        "count_mismatches": int(np.sum(f["nc"][deep] != nc[deep])),
        "rho_max_rel": float(np.max(np.abs(f["rho"][deep] - rho[deep]) / rho[deep])),
        "p_max_rel": float(np.max(np.abs(f["p"][deep] - P[deep]) / P[deep])),
        "accel_normwise": float(np.max(da) / np.max(np.linalg.norm(a_ref, axis=1))),
        "accel_max_over_sum_abs_terms": float(np.max(da / amag[deep])),
        "du_max_over_sum_abs_terms":
            float(np.max(np.abs(f["du"][deep] - du[deep]) / (dumag[deep] + 1e-300))),
        "divv_max_over_sum_abs_terms":
            float(np.max(np.abs(f["divv"][deep] - divv[deep]) / (dvmag[deep] + 1e-300))),
        "tolerance": tol,
        "oracle_s": round(t_oracle, 3),
    }
    out["within_tolerance"] = bool(
        out["count_mismatches"] == 0 and out["rho_max_rel"] <= tol
        and out["accel_max_over_sum_abs_terms"] <= tol and out["du_max_over_sum_abs_terms"] <= tol)
    return out


def _time_oracle(O, ic, steps, threads):
    O.set_num_threads(threads)
    st = O.State(ic, O.Params())
    st.evaluate(method=1)
    t0 = time.perf_counter()
    for _ in range(steps):
        st.step(None, method=1)
    return time.perf_counter() - t0


def cpu_baseline(config, samples, params_kw):
    """The oracle as it stands: (1) the accuracy of each timed GPU form on
    its cube sample; (2) the oracle's own throughput on a cut of the
    benchmark workload (the same lattice spacing, jitter, velocity field and
    energy, hence the same work per particle), all host threads and one."""
    import oracle as O
    from paper_1905_03344_amd import inputs
    acc = {}
    nthreads = os.cpu_count() or 1
    O.set_num_threads(nthreads)
    for form, f in samples.items():
        if f is not None:
            log(f"bench: oracle accuracy check of {form} ({len(f['x'])} particles)")
            acc[form] = _accuracy(O, f, params_kw)
    seed = inputs.CONFIG_SEEDS[config]
    if config == 4:
        ic_all = inputs.clumpy(n_clumps=16, per_clump=12500, n_background=50000, seed=seed)
        ic_one = inputs.clumpy(n_clumps=4, per_clump=2500, n_background=2500, seed=seed)
        cut = "clumpy mixture cut to {n} particles (16 / 4 clumps)"
        steps_all, steps_one = 2, 2
    else:
        s = {1: 1 / 20, 2: 1 / 100, 3: 1 / 200, 5: 1 / 400}[config]
        ic_all = inputs.square_patch(64, seed, spacing=s)
        ic_one = inputs.square_patch(32, seed, spacing=s)
        cut = f"{{side}}^3 = {{n}}-particle cut of the square patch at its spacing {s:g}"
        steps_all, steps_one = 3, 4
    log(f"bench: oracle timing, {nthreads} threads, n={ic_all.n}")
    t_all = _time_oracle(O, ic_all, steps_all, nthreads)
    log(f"bench: oracle timing, 1 thread, n={ic_one.n}")
    t_one = _time_oracle(O, ic_one, steps_one, 1)
    O.set_num_threads(nthreads)

    def desc(ic, steps, t, side):
        return (f"{steps} KDK steps (Courant dt) of a " + cut.format(side=side, n=ic.n)
                + f" after an untimed t=0 evaluation, {t:.2f} s")
    rec = {"value": ic_all.n * steps_all / t_all, "unit": "particle-updates/s",
           "cores": nthreads, "kind": "oracle",
           "sample": desc(ic_all, steps_all, t_all, 64),
           "single_thread": {"value": ic_one.n * steps_one / t_one, "cores": 1,
                             "sample": desc(ic_one, steps_one, t_one, 32)},
           "host": host_info()}
    return rec, acc


# ---------------------------------------------------------------------------
def _kernel_roofline(rec, n):
    """Achieved algorithmic rates of the walk and the pair kernels from the
    live stage timings (HIP events around each launch on the bound stream)."""
    wk = rec["work_per_step"]
    pairs_l, pairs = wk["pairs_L"], wk["pairs_S"]
    work = {
        "k_hsolve_round": (HSOLVE_FLOPS_PER_CANDIDATE * HSOLVE_CANDIDATES_PER_PARTICLE * n,
                           HWALK_BYTES_PER_PARTICLE * n + 4 * pairs_l),
        "k_forces": (FORCE_FLOPS_PER_PAIR * pairs,
                     FORCE_BYTES_PER_PARTICLE * n + FORCE_BYTES_PER_ENTRY * pairs),
        "k_density": (DENSITY_FLOPS_PER_PAIR * pairs_l,
                      DENSITY_BYTES_PER_PARTICLE * n + 4 * pairs_l),
    }
    kernels = {}
    for kname, (flops, nbytes) in work.items():
        t = rec["stages_ms_per_step"][KERNELS[kname][0]] * 1e-3
        tf = flops / t / 1e12 if t else 0.0
        gbs = nbytes / t / 1e9 if t else 0.0
        kernels[kname] = {"launch_ms": round(t * 1e3, 4), "flops_per_launch": int(flops),
                          "achieved_tflops": round(tf, 3),
                          "frac_fp64": round(tf / FP64_PEAK_TFLOPS, 4),
                          "algorithmic_bytes": int(nbytes), "achieved_gbs": round(gbs, 1),
                          "frac_hbm": round(gbs / HBM_PEAK_GBS, 4)}
    return kernels


def _roofline(kernels, workload):
    """The roofline object of the longest launch of the step."""
    dom = max(kernels, key=lambda k: kernels[k]["launch_ms"])
    kd = kernels[dom]
    traffic = profile_record(dom, workload, "traffic")
    counters = profile_record(dom, workload, "counters")
    # the bound the committed counter summary found for this kernel (VALU,
    # TA or HBM busiest); the arithmetic roofline when there is none
    bound = counters.get("bound", "alu") if counters else "alu"
    if bound == "hbm":
        achieved, peak, unit, frac = kd["achieved_gbs"], HBM_PEAK_GBS, "GB/s", kd["frac_hbm"]
    else:
        bound = "alu"
        achieved, peak, unit, frac = (kd["achieved_tflops"], FP64_PEAK_TFLOPS, "TFLOP/s",
                                      kd["frac_fp64"])
    return {"bound": bound, "kernel": dom, "achieved": achieved, "peak": peak, "unit": unit,
            "frac": frac,
            "traffic": traffic.get("bytes_per_launch") if traffic else None,
            "flops_per_launch": kd["flops_per_launch"], "launch_ms": kd["launch_ms"],
            "hbm": {"algorithmic_bytes": kd["algorithmic_bytes"], "achieved": kd["achieved_gbs"],
                    "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": kd["frac_hbm"]},
            "fp64": {"achieved": kd["achieved_tflops"], "peak": FP64_PEAK_TFLOPS,
                     "unit": "TFLOP/s", "frac": kd["frac_fp64"]},
            "counters": ({k: counters[k] for k in ("valu_busy", "ta_busy", "mfma_busy",
                                                   "hbm_frac_measured") if k in counters}
                         if counters else None)}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--config", type=int, default=5, choices=sorted(CONFIG_NAMES))
    ap.add_argument("--form", default="headline",
                    choices=["headline", "plain", "mixed", "learned"],
                    help="headline: plain FP64 and mixed + learned h on the same input")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--search-div", type=int, default=2)
    ap.add_argument("--max-level", type=int, default=None,
                    help="finest cell level of the search table (default: from n and h)")
    ap.add_argument("--integrator", default="kdk", choices=["kdk", "ab2"],
                    help="kick-drift-kick, or its positions with Adams-Bashforth energy")
    ap.add_argument("--gradients", default="kernel", choices=["kernel", "iad"],
                    help="gradient estimator of the momentum and energy sums")
    ap.add_argument("--walk-defer-group", type=int, default=None,
                    help="first-round walk sub-groups up to this size go to the per-particle "
                         "tail (default: 16 on the clumpy mixture, else the library's 4)")
    ap.add_argument("--grad-h", action="store_true",
                    help="grad-h correction terms in the momentum and energy sums")
    ap.add_argument("--kernel", default="m4", choices=["m4", "wendland", "sinc5"],
                    help="smoothing kernel of the density and force sums")
    ap.add_argument("--walk-prefilter", default="matrix", choices=["matrix", "none"],
                    help="candidate test of the h-iteration walk: bf16 Gram prefilter on the "
                         "matrix cores with an exact FP64 band, or FP64 for every candidate")
    ap.add_argument("--walk-strategy", default="auto", choices=["auto", "shell", "worklist"],
                    help="after the first count: the shell of that count (small runs) or a "
                         "worklist round (large runs); auto picks by size")
    ap.add_argument("--learned-try-shell", default="auto", choices=["auto", "never", "always"],
                    help="shell of the learned form's try (speed only): auto records the plain "
                         "count's shell where many tries miss in runs under 4M particles")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a 1 GiB device copy (PMC byte-counter calibration)")
    args = ap.parse_args()
    if args.copy_calibration:
        copy_calibration()
        return
    if args.gpus != 1:
        print(f"bench.py measures one GPU only (got --gpus {args.gpus}): the library runs the "
              "hot path on a single GPU; the sharded multi-GPU path is a design, not code",
              file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1905_03344_amd import ffi, inputs

    torch.cuda.init()
    args.prefilter = (ffi.SPH_PREFILTER_MATRIX if args.walk_prefilter == "matrix"
                      else ffi.SPH_PREFILTER_NONE)
    args.kernel_id = {"m4": ffi.SPH_KERNEL_M4, "wendland": ffi.SPH_KERNEL_WENDLAND,
                      "sinc5": ffi.SPH_KERNEL_SINC5}[args.kernel]
    args.integrator_id = (ffi.SPH_INTEGRATOR_AB2 if args.integrator == "ab2"
                          else ffi.SPH_INTEGRATOR_KDK)
    args.gradients_id = (ffi.SPH_GRADIENTS_IAD if args.gradients == "iad"
                         else ffi.SPH_GRADIENTS_KERNEL)
    args.strategy_id = {"auto": ffi.SPH_WALK_AUTO, "shell": ffi.SPH_WALK_SHELL_FIRST,
                        "worklist": ffi.SPH_WALK_WORKLIST}[args.walk_strategy]
    args.try_shell_id = {"auto": ffi.SPH_TRY_SHELL_AUTO, "never": ffi.SPH_TRY_SHELL_NEVER,
                         "always": ffi.SPH_TRY_SHELL_ALWAYS}[args.learned_try_shell]
    config = args.config
    # complement rows: the clumpy mixture's density contrast needs more slots
    extra_slots = 96 if config == 4 else 48
    defer = args.walk_defer_group
    if defer is None:
        defer = 16 if config == 4 else 0
    forms = {"headline": ["plain", "learned"], "plain": ["plain"], "mixed": ["mixed"],
             "learned": ["learned"]}[args.form]
    # the learned form is evaluated on seed B of the workload after training
    # on plain steps of seed A (the same distribution); in the headline both
    # forms run on seed B, so that they see the same input
    seed_b = "learned" in forms
    log(f"bench: config {config}, forms {forms}, building inputs")
    ic = inputs.config_ic(config, seed_offset=100 if seed_b else 0)
    n = ic.n
    records, samples = {}, {}
    want = not args.no_cpu_baseline
    if "plain" in forms:
        records["plain"], samples["plain"] = run_form(args, config, "plain", ic, False,
                                                      defer=defer, extra_slots=extra_slots,
                                                      want_sample=want)
    if "mixed" in forms:
        records["mixed"], samples["mixed"] = run_form(args, config, "mixed", ic, True,
                                                      defer=defer, extra_slots=extra_slots,
                                                      want_sample=want)
    training = None
    if "learned" in forms:
        ic_b = ic
        del ic
        ic_a = inputs.config_ic(config)
        log("bench: learned: harvesting and training on seed A")
        weights, training = train_learned(args, config, ic_a, defer, extra_slots)
        del ic_a
        records["learned"], samples["learned"] = run_form(args, config, "mixed+learned", ic_b,
                                                          True, learned_weights=weights,
                                                          defer=defer, extra_slots=extra_slots,
                                                          want_sample=want)
        records["learned"]["training"] = training
        del ic_b
    else:
        del ic

    main_form = forms[0]
    main = records[main_form]
    workload = CONFIG_NAMES[config]
    kernels = _kernel_roofline(main, n)
    out = {
        "metric": "particle-updates/s per full SPH step",
        "value": main["value"],
        "unit": "particle-updates/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": main["ms_per_step"],
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64" if main_form == "plain" else "f32",
        "data": "synthetic",
        "config": {"workload": workload, "n": n,
                   "seed": inputs.CONFIG_SEEDS[config] + (100 if seed_b else 0),
                   "form": main_form, "dt": "courant cfl 0.3",
                   "walk_prefilter": args.walk_prefilter, "walk_defer_group": defer or 4,
                   "walk_strategy": args.walk_strategy,
                   "learned_try_shell": args.learned_try_shell,
                   "kernel": args.kernel, "integrator": args.integrator,
                   "grad_h": bool(args.grad_h), "gradients": args.gradients},
        "roofline": _roofline(kernels, workload) if main_form == "plain" else None,
        "kernels": kernels,
        "stages_ms_per_step": main["stages_ms_per_step"],
        "work_per_step": main["work_per_step"],
        "forms": records,
        "status": main["status"],
    }
    if main_form != "plain":
        # the mixed-form kernels are timed in the same stages; their FP32
        # work priced against the FP64 peak would not be a roofline
        out["roofline"] = {"bound": "alu", "kernel": max(kernels,
                                                         key=lambda k: kernels[k]["launch_ms"]),
                           "achieved": None, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                           "frac": None, "traffic": None}
    if "plain" in records and "learned" in records:
        records["learned"]["speedup_over_plain_fp64"] = (records["plain"]["ms_per_step"]
                                                        / records["learned"]["ms_per_step"])
    if want:
        log("bench: cpu baseline (oracle)")
        params_kw = {"kernel": args.kernel_id, "grad_h": bool(args.grad_h),
                     "iad": args.gradients == "iad"}
        out["cpu_baseline"], acc = cpu_baseline(config, samples, params_kw)
        for form, a in acc.items():
            records[form]["accuracy"] = a
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
