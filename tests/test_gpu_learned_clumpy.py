"""The learned smoothing length on the clumpy mixture, where h varies ~10x:
what the trained network gains over the plain iteration, and parity of the
learned step against the oracle at its own h.

* Gain (1,000,000 particles, the clumpy workload's size and recipe): a
  model trained on 20 plain steps of seed A is run on seed B (the same
  distribution) next to the plain iteration and next to a zero model (its
  try is h_prev itself), in the mixed form with the clumpy workload's walk
  settings (centred targets, deferral of sub-groups up to 16).  Counted per
  step: neighbour counts per particle, candidates tested by the walks,
  fallback rate, and the h iteration's time (with and without the MLP's,
  for the learned form).  Counts, candidates and fallbacks are exact and
  asserted; so is the first walk's time (the accepted try is counted
  without the shell the plain count records: ~15% less).  The h iteration
  as a whole is level with the plain one on this workload (the walk's
  saving goes to the per-particle tail that serves the 0.6% of misses:
  2.49 against 2.56 ms measured, 2.60 with the MLP's inference), so its time
  is asserted within 5% of plain's, and reported.
* Parity (125,000 particles, one learned step from the oracle's state):
  cells, counts and both neighbour sets exact, accepted h in band by the
  oracle's count, fallback h identical to the plain iteration's, fields at
  the learned form's own h within the mixed form's tolerance; plus a sampled
  cube of the 1M gain run against the oracle at its own h.

Set SPH_TEST_REPORT to a file name to have the gain figures written there
as JSON."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs

pytestmark = pytest.mark.gpu

DEFER = 16
EXTRA = 96


def _clumpy_1m(seed):
    return inputs.clumpy(seed=seed)


def _clumpy_125k(seed):
    return inputs.clumpy(n_clumps=8, per_clump=12500, n_background=25000, seed=seed)


def _train(ic, steps, seed):
    from paper_1905_03344_amd import ffi, learned
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(ic, precision=ffi.SPH_MIXED, extra_per_particle=EXTRA,
                     walk_defer_group=DEFER)
    sim.evaluate()
    feat, target = learned.harvest(sim, steps=steps, target_mode=ffi.SPH_TARGET_CENTRED)
    sim.sync()
    w, norm, losses = learned.train(sim, feat, target, seed=seed)
    zero_mse = float((target.double() ** 2).mean())
    del feat, target, sim
    return w, norm, losses, zero_mse


def _measure(ic, h_mode, w=None, norm=None, warmup=2, steps=5):
    import torch
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(ic, precision=ffi.SPH_MIXED, h_mode=h_mode, extra_per_particle=EXTRA,
                     walk_defer_group=DEFER)
    if w is not None:
        sim.set_mlp(w, norm)
    sim.evaluate()
    for _ in range(warmup):
        sim.step(0.0)
    sim.sync()
    ffi.sph_timing(sim.ctx, True)
    counts = cand = acc = fb = 0
    for _ in range(steps):
        sim.step(0.0)
        _, st = sim.sync()
        counts += st.h_counts
        cand += st.candidates
        acc += st.learned_accepted
        fb += st.learned_fallback
    stages = ffi.sph_timing_read(sim.ctx)
    ffi.sph_timing(sim.ctx, False)
    torch.cuda.synchronize()
    n = sim.n
    dec = acc + fb
    rec = {"counts_per_particle": counts / steps / n,
           "candidates_per_particle": cand / steps / n,
           "hsolve_ms": stages["hsolve"][0] / steps,
           "walk_ms": stages["hwalk"][0] / steps,
           "mlp_ms": stages["mlp"][0] / steps,
           "step_ms": sum(v[0] for k, v in stages.items() if k != "hwalk") / steps,
           "fallback_rate": fb / dec if dec else None}
    rec["hsolve_total_ms"] = rec["hsolve_ms"] + rec["mlp_ms"]
    return sim, rec


@pytest.fixture(scope="module")
def trained_1m():
    seed = inputs.CONFIG_SEEDS[4]
    w, norm, losses, zero_mse = _train(_clumpy_1m(seed), 20, seed)
    return w, norm, losses, zero_mse


def test_learned_gain_clumpy_1m(trained_1m):
    from paper_1905_03344_amd import ffi
    from test_gpu_fullsize import _sampled_check
    w, norm, losses, zero_mse = trained_1m
    ic_b = _clumpy_1m(inputs.CONFIG_SEEDS[4] + 100)
    _, plain = _measure(ic_b, ffi.SPH_H_PLAIN)
    wz = {k: v.copy() for k, v in w.items()}
    wz["W3"][:] = 0.0
    wz["b3"][:] = 0.0
    _, zero = _measure(ic_b, ffi.SPH_H_LEARNED, wz, norm)
    sim, learned = _measure(ic_b, ffi.SPH_H_LEARNED, w, norm)
    report = {"n": ic_b.n, "plain": plain, "zero_model": zero, "learned": learned,
              "training": {"loss_first": float(losses[0]), "loss_last": float(losses[-1]),
                           "target_mse_zero_model": zero_mse}}
    print(json.dumps(report), flush=True)
    path = os.environ.get("SPH_TEST_REPORT")
    if path:
        with open(path, "w") as f:
            json.dump(report, f, indent=1)
    # the trained model is far better than predicting no change
    assert float(np.mean(losses[-50:])) < 0.5 * zero_mse
    # fewer counts than the plain iteration and than a try at h_prev, and
    # fewer fallbacks than the try at h_prev (about half; h_prev is already
    # in band for ~98% of the particles, so the plain solve takes ~1.02
    # counts)
    assert learned["counts_per_particle"] < plain["counts_per_particle"]
    assert learned["counts_per_particle"] < zero["counts_per_particle"]
    assert learned["fallback_rate"] < 0.75 * zero["fallback_rate"]
    assert learned["fallback_rate"] < 0.05
    # fewer candidates and less time in the first walk (the accepted try is
    # counted without the shell the plain count records); the h iteration as
    # a whole level with plain's
    assert learned["candidates_per_particle"] < plain["candidates_per_particle"]
    assert learned["walk_ms"] < 0.95 * plain["walk_ms"]
    assert learned["hsolve_ms"] < 1.05 * plain["hsolve_ms"]
    # the learned run itself, sampled against the oracle at its own h
    # a cube about the densest clump, kept inside [0.1, 0.9]^3 where the
    # background bounds h (outside the unit cube only sparse clump tails
    # remain, with h up to ~1)
    h = sim.field("h")
    k = int(h.argmin())
    c = tuple(min(max(float(sim.field(a)[k]), 0.25), 0.75) for a in ("x", "y", "z"))
    n = _sampled_check(sim, 1e-5, half=0.15, centre=c)
    print(f"learned clumpy 1M: {n} sampled particles agree", flush=True)


@pytest.fixture(scope="module")
def trained_125k():
    w, norm, losses, zero_mse = _train(_clumpy_125k(1905033454), 10, 1905033455)
    return w, norm


@pytest.mark.parametrize("strategy", ["auto", "worklist"])
def test_learned_step_clumpy_vs_oracle(trained_125k, strategy):
    """One learned step of the mixed form on a 125,000-particle clumpy set
    (seed B) from the oracle's state, with the clumpy workload's settings;
    misses restart in the per-particle tail (auto at this size) or in a
    worklist round first."""
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation
    from test_gpu_mixed import check_mixed_fields
    from test_gpu_parity import _upload_oracle_state, compare_cells, compare_neighbors
    w, norm = trained_125k
    ic = _clumpy_125k(1905033554)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    sim = Simulation(ic, h_mode=ffi.SPH_H_LEARNED, precision=ffi.SPH_MIXED,
                     extra_per_particle=EXTRA, walk_defer_group=DEFER,
                     walk_strategy=(ffi.SPH_WALK_WORKLIST if strategy == "worklist"
                                    else ffi.SPH_WALK_AUTO))
    sim.set_mlp(w, norm)
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    plain = O.State(ic.copy())
    plain.f = {k: v.copy() for k, v in st.f.items()}
    plain.step(dt, method=1)
    sim.step(dt)
    code, stats = sim.sync()
    h = sim.numpy("h")
    flags = sim.numpy("flags")
    acc = (flags & ffi.SPH_FLAG_LEARNED) != 0
    print(f"learned clumpy 125k: accepted {acc.mean():.3f}", flush=True)
    assert stats.learned_accepted == int(acc.sum())
    assert stats.learned_accepted + stats.learned_fallback == ic.n
    assert acc.mean() > 0.8
    np.testing.assert_array_equal(h[~acc], plain.f["h"][~acc])
    st.h_given = h
    st.step(dt, method=1)
    compare_cells(sim, st)
    np.testing.assert_array_equal(sim.numpy("nc"), st.f["nc"])
    assert np.all(np.abs(st.f["nc"][acc] - 100) <= 5)
    compare_neighbors(sim, st)
    check_mixed_fields(sim, st)
