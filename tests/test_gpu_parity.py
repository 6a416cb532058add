"""GPU parity of the plain FP64 path against the CPU oracle, through the C ABI.

Both sides start from the same seeded inputs; nothing computed on the GPU is
ever fed to the oracle.  Integer and index results (bounding box, keys,
permutation, cell table, h, counts, flags, gather sets L_i, complement rows
E_i) must match bit for bit; FP64 fields within 1e-12 relative, signed sums
(divergence, acceleration, du) within 1e-12 of the oracle's sum of term
magnitudes (the conditioning of each sum)."""
import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _sim(ic, **kw):
    from paper_1905_03344_amd.state import Simulation
    return Simulation(ic, **kw)


def _pairs(n, rows_len, cols):
    rows = np.repeat(np.arange(n, dtype=np.int64), rows_len)
    return rows * n + cols.astype(np.int64)


def gpu_gather_codes(sim):
    nc, idx = sim.gather_dense()
    n = sim.n
    K = idx.shape[0]
    mask = np.arange(K)[:, None] < np.minimum(nc, K)[None, :]
    kk, ii = np.nonzero(mask)
    return np.sort(ii.astype(np.int64) * n + idx[kk, ii].astype(np.int64))


def compare_cells(sim, st):
    np.testing.assert_array_equal(sim.numpy("perm"), st.perm)
    np.testing.assert_array_equal(sim.numpy("key"), st.keys)
    np.testing.assert_array_equal(sim.numpy("id"), st.f["id"])
    bb = sim.bbox()
    np.testing.assert_array_equal(bb[:3], st.lo)
    np.testing.assert_array_equal(bb[3:], st.hi)
    table = sim.cell_table()
    np.testing.assert_array_equal(table, O.cell_start(st.keys, sim.params.max_level))
    for f in ("x", "y", "z", "m"):
        np.testing.assert_array_equal(sim.numpy(f), st.f[f])


def compare_neighbors(sim, st):
    n = sim.n
    np.testing.assert_array_equal(sim.numpy("h"), st.f["h"])
    np.testing.assert_array_equal(sim.numpy("nc"), st.f["nc"])
    np.testing.assert_array_equal(sim.numpy("flags") & 1, st.flags)
    # gather sets as sets
    ref_l = _pairs(n, np.diff(st.loff), st.lidx)
    np.testing.assert_array_equal(gpu_gather_codes(sim), ref_l)
    # complement rows, ascending, exactly
    ref_s = _pairs(n, np.diff(st.off), st.idx)
    ref_e = np.setdiff1d(ref_s, ref_l, assume_unique=True)
    eoff, eidx = sim.extra_lists()
    ecount = np.bincount((ref_e // n).astype(np.int64), minlength=n)
    np.testing.assert_array_equal(eoff, np.concatenate([[0], np.cumsum(ecount)]))
    np.testing.assert_array_equal(eidx, (ref_e % n).astype(np.int32))


def rel_err(a, b):
    return np.max(np.abs(a - b) / np.maximum(np.abs(b), 1e-300)) if len(a) else 0.0


def compare_fields(sim, st):
    assert rel_err(sim.numpy("rho"), st.f["rho"]) <= TOL
    dv = np.abs(sim.numpy("divv") - st.f["divv"])
    assert np.all(dv <= TOL * (st.divv_mag + 1e-300)), np.max(dv / (st.divv_mag + 1e-300))
    assert rel_err(sim.numpy("p"), st.P) <= TOL
    assert rel_err(sim.numpy("c"), st.c) <= TOL
    for k in ("ax", "ay", "az"):
        d = np.abs(sim.numpy(k) - st.f[k])
        assert np.all(d <= TOL * st.amag + 1e-300), (k, np.max(d / (st.amag + 1e-300)))
        ref = np.max(np.abs(st.f[k]))
        assert np.max(d) <= TOL * max(ref, 1e-300) * 10
    d = np.abs(sim.numpy("du") - st.f["du"])
    assert np.all(d <= TOL * st.dumag + 1e-300), np.max(d / (st.dumag + 1e-300))
    assert abs(sim.dt() - st.dt_next) <= TOL * st.dt_next


CASES = {
    "patch_20^3": lambda: inputs.square_patch(20, inputs.CONFIG_SEEDS[1]),
    "patch_23^3_ragged": lambda: inputs.square_patch(23, 77),
    "clumpy_12k": lambda: inputs.clumpy(n_clumps=4, per_clump=2500, n_background=2000, seed=5),
}


@pytest.mark.parametrize("case", sorted(CASES))
def test_evaluate_parity(case):
    ic = CASES[case]()
    print(f"case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96)
    sim.evaluate()
    code, stats = sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    assert stats.nonconverged == st.nonconv
    assert stats.extra_total == st.off[-1] - st.loff[-1]


def test_stage_calls_parity():
    ic = inputs.square_patch(18, 3)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic)
    sim.build_cells()
    compare_cells(sim, st)
    sim.copy_pred_from_state()
    sim.find_neighbors()
    compare_neighbors(sim, st)
    sim.density()
    sim.eos()
    sim.momentum_energy()
    sim.sync()
    compare_fields(sim, st)


def _upload_oracle_state(sim, st):
    for f in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u", "ax", "ay", "az", "du", "rho", "divv"):
        sim.set_field(f, st.f[f])
    sim.set_field("nc", st.f["nc"].astype(np.int32))
    sim.set_field("id", st.f["id"].astype(np.int32))


@pytest.mark.parametrize("dt", [1e-4, 0.0])
def test_step_parity(dt):
    ic = inputs.square_patch(20, inputs.CONFIG_SEEDS[1])
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic)
    _upload_oracle_state(sim, st)
    sim.d_dt.fill_(st.dt_next)
    st.step(dt if dt > 0 else None, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    for f in ("vx", "vy", "vz", "u"):
        scale = np.max(np.abs(st.f[f]))
        assert np.max(np.abs(sim.numpy(f) - st.f[f])) <= TOL * scale


def test_ab2_step_parity():
    """The Adams-Bashforth energy integrator: an Euler first step and an AB2
    second step with a different dt, each from the oracle's state."""
    from paper_1905_03344_amd import ffi
    ic = inputs.square_patch(20, inputs.CONFIG_SEEDS[1])
    st = O.State(ic.copy(), O.Params(integrator=O.INTEGRATOR_AB2))
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, integrator=ffi.SPH_INTEGRATOR_AB2)
    sim.evaluate()
    for k, dt in enumerate((1e-4, 1.5e-4)):
        _upload_oracle_state(sim, st)
        st.step(dt, method=1)
        sim.step(dt)
        sim.sync()
        compare_cells(sim, st)
        compare_neighbors(sim, st)
        compare_fields(sim, st)
        for f in ("vx", "vy", "vz", "u"):
            scale = np.max(np.abs(st.f[f]))
            assert np.max(np.abs(sim.numpy(f) - st.f[f])) <= TOL * scale, (k, f)


@pytest.mark.parametrize("case", ["patch_21^3", "clumpy_12k"])
def test_conservation_parity(case):
    """All seven sums: E relative, P normalised by sum m|v| and every
    component of L by sum m|x||v| (the patch's P, L_x and L_y vanish
    analytically; the clumpy set's noisy velocities make all seven
    non-trivial)."""
    ic = (inputs.square_patch(21, 9) if case == "patch_21^3"
          else inputs.clumpy(n_clumps=4, per_clump=2500, n_background=2000, seed=5))
    st = O.State(ic.copy())
    sim = _sim(ic, extra_per_particle=96)
    out = sim.conservation()
    ref = st.conservation()
    assert abs(out[6] - ref[6]) <= TOL * abs(ref[6])
    vmag = np.sqrt(ic.vx ** 2 + ic.vy ** 2 + ic.vz ** 2)
    pscale = np.sum(ic.m * vmag)
    lscale = np.sum(ic.m * np.sqrt(ic.x ** 2 + ic.y ** 2 + ic.z ** 2) * vmag)
    assert np.all(np.abs(out[:3] - ref[:3]) <= TOL * pscale), (out[:3], ref[:3])
    assert np.all(np.abs(out[3:6] - ref[3:6]) <= TOL * lscale), (out[3:6], ref[3:6])
    if case == "patch_21^3":
        assert abs(out[5] - ref[5]) <= TOL * abs(ref[5])
    else:
        assert np.all(np.abs(ref[3:6]) > 1e-6 * lscale)


def test_deterministic_runs():
    ic = inputs.clumpy(n_clumps=3, per_clump=2000, n_background=1500, seed=21)
    outs = []
    for _ in range(2):
        sim = _sim(ic, extra_per_particle=96)
        sim.evaluate()
        for _ in range(2):
            sim.step(0.0)
        sim.sync()
        outs.append({f: sim.numpy(f).copy() for f in ("x", "vx", "h", "rho", "ax", "du", "nc")})
    for f in outs[0]:
        np.testing.assert_array_equal(outs[0][f], outs[1][f])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_complement_order_paths(precision):
    """Complement rows ranked inside the force kernel (row capacity up to
    128) and rows sorted in memory first (larger capacity) are visited in the
    same ascending order, so the sums agree bit for bit."""
    from paper_1905_03344_amd import ffi
    ic = inputs.clumpy(n_clumps=3, per_clump=2000, n_background=1500, seed=21)
    prec = ffi.SPH_FP64 if precision == "fp64" else ffi.SPH_MIXED
    outs = []
    for slots in (96, 160):
        sim = _sim(ic, extra_per_particle=slots, precision=prec)
        sim.evaluate()
        sim.step(0.0)
        sim.sync()
        assert int((sim.nl_ecnt[:sim.n] > 16).sum()) > 100   # rows that span several lane rounds
        outs.append({f: sim.numpy(f).copy() for f in ("ax", "ay", "az", "du", "x", "u")})
    for f in outs[0]:
        np.testing.assert_array_equal(outs[0][f], outs[1][f])


@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_walk_prefilter_paths(case):
    """The matrix-core prefilter of the walk tiles and the plain FP64 test of
    every candidate give the same gather sets (in the same order), shells,
    h and fields, bit for bit, after an evaluation and a step."""
    from paper_1905_03344_amd import ffi
    ic = CASES[case]()
    outs = []
    for pf in (ffi.SPH_PREFILTER_NONE, ffi.SPH_PREFILTER_MATRIX):
        print(f"walk paths {case} prefilter {pf}", flush=True)
        sim = _sim(ic, extra_per_particle=96, walk_prefilter=pf)
        sim.evaluate()
        sim.step(0.0)
        sim.sync()
        nc, idx = sim.gather_dense()
        out = {f: sim.numpy(f).copy() for f in ("h", "nc", "rho", "ax", "ay", "az", "du", "x")}
        used = np.arange(idx.shape[0])[:, None] < np.minimum(nc, idx.shape[0])[None, :]
        out["lists"] = np.where(used, idx, -1)
        outs.append(out)
    for f in outs[0]:
        np.testing.assert_array_equal(outs[0][f], outs[1][f], err_msg=f)


@pytest.mark.parametrize("defer", [16, 64])
@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_walk_defer_group_parity(case, defer):
    """More of the first round left to the per-particle tail: the same cells,
    sets, h and counts as the oracle, fields to the usual tolerance (a gather
    row may come in another order), after an evaluation and a step."""
    ic = CASES[case]()
    print(f"walk defer {defer} case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96, walk_defer_group=defer)
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    st.step(dt, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)


def _gather_rows_flat(sim):
    """The gather rows concatenated in particle order, each in stored order."""
    nc, idx = sim.gather_dense()
    K = idx.shape[0]
    mask = np.arange(K)[:, None] < np.minimum(nc, K)[None, :]
    return idx.T[mask.T]


@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_gather_rows_canonical_and_csr(case):
    """Every gather row L_i is stored in ascending index order, so it equals
    the oracle's row element by element (not only as a set), whether the
    walk counted it in a group, completed it from a shell, or left it to the
    per-particle tail: with walk_defer_group 4, 16 and 64, and with the
    first count recording its shell or leaving the misses to a worklist
    round, the rows and every field are bit-identical after an evaluation
    and a step.  The CSR export of S_i = L_i U E_i equals the oracle's
    interaction sets exactly."""
    from paper_1905_03344_amd import ffi
    ic = CASES[case]()
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    st0 = {k: v.copy() for k, v in st.f.items()}
    dt = st.dt_next
    ref_rows_t0 = st.lidx.copy()
    st.step(dt, method=1)
    outs = []
    for defer, strategy in ((0, ffi.SPH_WALK_AUTO), (16, ffi.SPH_WALK_SHELL_FIRST),
                            (64, ffi.SPH_WALK_SHELL_FIRST), (0, ffi.SPH_WALK_WORKLIST),
                            (16, ffi.SPH_WALK_WORKLIST)):
        print(f"canonical rows {case} defer {defer} strategy {strategy}", flush=True)
        sim = _sim(ic, extra_per_particle=96, walk_defer_group=defer, walk_strategy=strategy)
        sim.evaluate()
        sim.sync()
        np.testing.assert_array_equal(_gather_rows_flat(sim), ref_rows_t0)
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u", "ax", "ay", "az", "du", "rho",
                  "divv"):
            sim.set_field(f, st0[f])
        sim.set_field("nc", st0["nc"].astype(np.int32))
        sim.set_field("id", st0["id"].astype(np.int32))
        sim.step(dt)
        sim.sync()
        compare_cells(sim, st)
        np.testing.assert_array_equal(sim.numpy("h"), st.f["h"])
        np.testing.assert_array_equal(sim.numpy("nc"), st.f["nc"])
        np.testing.assert_array_equal(_gather_rows_flat(sim), st.lidx)
        off, idx = sim.interaction_csr_device()
        np.testing.assert_array_equal(off.cpu().numpy(), st.off)
        np.testing.assert_array_equal(idx.cpu().numpy(), st.idx)
        outs.append({f: sim.numpy(f).copy() for f in ("rho", "divv", "ax", "ay", "az", "du")})
    for o in outs[1:]:
        for f in o:
            np.testing.assert_array_equal(outs[0][f], o[f], err_msg=f)


def test_interaction_csr_capacity():
    """Too small an index array: d_off complete, nothing written past the
    capacity, SPH_ECAPACITY from the next sync."""
    import torch
    from paper_1905_03344_amd import ffi
    ic = inputs.square_patch(12, 4)
    sim = _sim(ic)
    sim.evaluate()
    sim.sync()
    off, idx = sim.interaction_csr_device()
    total = int(off[-1])
    off2 = torch.zeros_like(off)
    buf = torch.full((total,), -7, dtype=torch.int32, device=sim.device)
    cap = total // 2
    ffi.sph_interaction_csr(sim.ctx, sim.s, sim.nl, off2.data_ptr(), buf.data_ptr(), cap)
    with pytest.raises(ffi.SphError) as e:
        sim.sync()
    assert e.value.code == ffi.SPH_ECAPACITY
    np.testing.assert_array_equal(off2.cpu().numpy(), off.cpu().numpy())
    b = buf.cpu().numpy()
    np.testing.assert_array_equal(b[:cap], idx.cpu().numpy()[:cap])
    assert np.all(b[cap:] == -7)


KERNEL_VARIANTS = ["wendland", "sinc5"]


def _kernel_id(name):
    from paper_1905_03344_amd import ffi
    return {"wendland": ffi.SPH_KERNEL_WENDLAND, "sinc5": ffi.SPH_KERNEL_SINC5}[name]


@pytest.mark.parametrize("kernel", KERNEL_VARIANTS)
@pytest.mark.parametrize("case", ["patch_20^3", "clumpy_12k"])
def test_kernel_variants_parity(case, kernel):
    """The kernel section's Wendland C2 and sinc kernels: an evaluation and a
    step from identical state against the oracle with the same kernel."""
    kid = _kernel_id(kernel)
    assert kid == {"wendland": O.KERNEL_WENDLAND, "sinc5": O.KERNEL_SINC5}[kernel]
    ic = CASES[case]()
    print(f"kernel {kernel} case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy(), O.Params(kernel=kid))
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96, kernel=kid)
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    st.step(dt, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)


@pytest.mark.parametrize("kernel", ["m4", "wendland"])
@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_grad_h_parity(case, kernel):
    """Grad-h correction terms: Omega, the forces and a step against the
    oracle with the same terms."""
    kid = {"m4": O.KERNEL_M4, "wendland": O.KERNEL_WENDLAND}[kernel]
    ic = CASES[case]()
    print(f"grad-h kernel {kernel} case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy(), O.Params(kernel=kid, grad_h=True))
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96, kernel=kid, grad_h=True)
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    om = sim.omega()
    assert np.max(np.abs(om - st.omega)) <= 10 * TOL
    assert np.max(np.abs(st.omega - 1.0)) > 1e-3   # the correction is not trivial
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    st.step(dt, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    assert np.max(np.abs(sim.omega() - st.omega)) <= 10 * TOL


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("kernel", ["m4", "wendland"])
@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_generalized_volumes_parity(case, kernel, precision):
    """Generalized volume elements (weights (m/rho)^0.7 of the previous
    density; the standard density first at t = 0): density, forces and a
    step from the oracle's state against the oracle with the same volumes,
    FP64 to 1e-12, the mixed form to its tolerance."""
    from paper_1905_03344_amd import ffi
    from test_gpu_mixed import check_mixed_fields
    kid = {"m4": O.KERNEL_M4, "wendland": O.KERNEL_WENDLAND}[kernel]
    ic = CASES[case]()
    print(f"volumes {precision} kernel {kernel} case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy(), O.Params(kernel=kid, volumes=O.VOLUMES_GENERALIZED,
                                     gve_exponent=0.7))
    st.keep_gather = True
    st.evaluate(method=1)
    prec = ffi.SPH_FP64 if precision == "fp64" else ffi.SPH_MIXED
    sim = _sim(ic, extra_per_particle=96, kernel=kid, precision=prec,
               volumes=ffi.SPH_VOLUMES_GENERALIZED, gve_exponent=0.7)
    check = compare_fields if precision == "fp64" else check_mixed_fields
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    check(sim, st)
    # a non-trivial change of the density against the standard volumes
    std = O.State(ic.copy(), O.Params(kernel=kid))
    std.evaluate(method=1)
    assert np.max(np.abs(st.f["rho"] / std.f["rho"] - 1.0)) > 1e-4
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    st.step(dt, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    check(sim, st)


def test_generalized_volumes_rejects_other_variants():
    from paper_1905_03344_amd import ffi
    for kw in ({"grad_h": True}, {"gradients": ffi.SPH_GRADIENTS_IAD}, {"gve_exponent": 1.5}):
        with pytest.raises(ffi.SphError):
            _sim(inputs.square_patch(6, 1), volumes=ffi.SPH_VOLUMES_GENERALIZED, **kw)


@pytest.mark.parametrize("variant", ["iad", "iad+grad_h", "iad_wendland"])
@pytest.mark.parametrize("case", ["patch_23^3_ragged", "clumpy_12k"])
def test_iad_parity(case, variant):
    """IAD gradients: the forces and a step against the oracle with the same
    estimator (and grad-h factors, or the Wendland kernel)."""
    from paper_1905_03344_amd import ffi
    kid = O.KERNEL_WENDLAND if variant == "iad_wendland" else O.KERNEL_M4
    gh = variant == "iad+grad_h"
    ic = CASES[case]()
    print(f"IAD variant {variant} case {case} n={ic.n}", flush=True)
    st = O.State(ic.copy(), O.Params(kernel=kid, grad_h=gh, gradients=O.GRADIENTS_IAD))
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96, kernel=kid, grad_h=gh,
               gradients=ffi.SPH_GRADIENTS_IAD)
    sim.evaluate()
    code, stats = sim.sync()
    assert stats.iad_singular == 0
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
    _upload_oracle_state(sim, st)
    dt = st.dt_next
    st.step(dt, method=1)
    sim.step(dt)
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)


def test_all_options_two_steps():
    """Every option at once -- Wendland kernel, IAD gradients, grad-h
    factors, the Adams-Bashforth energy update, no walk prefilter -- for two
    steps with different dt, each from the oracle's state."""
    from paper_1905_03344_amd import ffi
    ic = CASES["clumpy_12k"]()
    print(f"all options n={ic.n}", flush=True)
    st = O.State(ic.copy(), O.Params(kernel=O.KERNEL_WENDLAND, grad_h=True,
                                     gradients=O.GRADIENTS_IAD, integrator=O.INTEGRATOR_AB2))
    st.keep_gather = True
    st.evaluate(method=1)
    sim = _sim(ic, extra_per_particle=96, kernel=ffi.SPH_KERNEL_WENDLAND, grad_h=True,
               gradients=ffi.SPH_GRADIENTS_IAD, integrator=ffi.SPH_INTEGRATOR_AB2,
               walk_prefilter=ffi.SPH_PREFILTER_NONE)
    sim.evaluate()
    sim.sync()
    compare_fields(sim, st)
    for k, dt in enumerate((0.5 * st.dt_next, 0.8 * st.dt_next)):
        _upload_oracle_state(sim, st)
        st.step(dt, method=1)
        sim.step(dt)
        sim.sync()
        compare_cells(sim, st)
        compare_neighbors(sim, st)
        compare_fields(sim, st)
        for f in ("vx", "vy", "vz", "u"):
            scale = np.max(np.abs(st.f[f]))
            assert np.max(np.abs(sim.numpy(f) - st.f[f])) <= TOL * scale, (k, f)


def test_iad_singular_matrices_reported():
    """Two flat layers far apart (a three-dimensional box, but every
    neighbourhood lies in one plane): every IAD moment matrix is singular,
    which sph_sync reports as an error."""
    from paper_1905_03344_amd import ffi
    g = (np.arange(12) + 0.5) / 12
    x, y = (a.ravel() for a in np.meshgrid(g, g, indexing="ij"))
    x = np.concatenate([x, x])
    y = np.concatenate([y, y])
    z = np.concatenate([np.zeros(144), np.full(144, 10.0)])
    n = len(x)
    zeros = np.zeros(n)
    ic = inputs.ParticleSet(x, y, z, zeros.copy(), zeros.copy(), zeros.copy(), np.full(n, 1.0 / n),
                            np.full(n, 0.2), np.ones(n), name="two_layers")
    print(f"IAD singular layers n={ic.n}", flush=True)
    sim = _sim(ic, extra_per_particle=96, gradients=ffi.SPH_GRADIENTS_IAD)
    sim.evaluate()
    with pytest.raises(ffi.SphError) as e:
        sim.sync()
    assert e.value.code == ffi.SPH_ENONFINITE and "IAD" in str(e.value)


def test_lattice_nonconvergence_reported():
    from paper_1905_03344_amd import ffi
    ic = inputs.perfect_lattice(16)
    sim = _sim(ic)
    sim.evaluate()
    code, stats = sim.sync()
    assert code == ffi.SPH_WNOCONV
    assert stats.nonconverged == ic.n
    assert np.all(sim.numpy("nc") == 92)
    assert np.all(sim.numpy("flags") & 1)


def test_list_capacity_error_and_retry():
    from paper_1905_03344_amd import ffi
    ic = inputs.square_patch(16, 4)
    sim = _sim(ic, list_stride=64)
    sim.evaluate()
    with pytest.raises(ffi.SphError) as e:
        sim.sync()
    assert e.value.code == ffi.SPH_ECAPACITY
    sim2 = _sim(ic, list_stride=128)
    sim2.evaluate()
    code, _ = sim2.sync()
    assert code == ffi.SPH_OK


def test_tiny_inputs():
    # one particle: no neighbours, the iteration cannot converge
    ic = inputs.square_patch(4, 1).subset(np.array([5]))
    sim = _sim(ic)
    sim.evaluate()
    code, stats = sim.sync()
    assert stats.nonconverged == 1 and sim.numpy("nc")[0] == 0
    # empty set
    ic0 = inputs.square_patch(4, 1).subset(np.array([], dtype=np.int64))
    sim0 = _sim(ic0)
    sim0.evaluate()
    sim0.sync()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_coincident_particles(precision):
    """Particles at exactly the same position (with different velocities):
    each counts the other as a neighbour, the pair adds W(0) to the density
    and nothing to the gradient sums (the oracle skips r = 0 in the pair
    force; the kernels take 1/r as 0 there)."""
    from paper_1905_03344_amd import ffi
    from test_gpu_mixed import check_mixed_fields
    ic = inputs.square_patch(16, 9)
    rng = np.random.default_rng(4)
    src = rng.choice(ic.n, size=6, replace=False)
    for a, b in zip(src[:3], src[3:]):
        ic.x[b], ic.y[b], ic.z[b] = ic.x[a], ic.y[a], ic.z[a]
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    prec = ffi.SPH_FP64 if precision == "fp64" else ffi.SPH_MIXED
    sim = _sim(ic, extra_per_particle=96, precision=prec)
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    if precision == "fp64":
        compare_fields(sim, st)
    else:
        check_mixed_fields(sim, st)


def test_sort_of_scattered_keys_repeated():
    """The radix sort on a million keys in generator order (every digit pass
    moves nearly every key across its tile), on fresh states three times:
    the permutation equals the oracle's stable sort each time.  The scatter
    ranks a tile's keys into LDS round by round; a missing barrier between
    its rounds once let a wave clear the round counts another wave still read,
    which showed as an unsorted key at 8M particles."""
    ic = inputs.clumpy(seed=inputs.CONFIG_SEEDS[4])
    lo, hi = O.bbox(ic.x, ic.y, ic.z, ic.periodic, ic.box_lo, ic.box_hi)
    key = O.cell_keys(ic.x, ic.y, ic.z, lo, hi)
    perm = O.sort_perm(key)
    assert np.mean(perm != np.arange(ic.n)) > 0.99
    for rep in range(3):
        print(f"sort of scattered keys, repeat {rep}", flush=True)
        sim = _sim(ic)
        sim.build_cells()
        sim.sync()
        np.testing.assert_array_equal(sim.numpy("perm"), perm)
        np.testing.assert_array_equal(sim.numpy("key"), key[perm])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("variant", ["grad_h", "iad"])
def test_tiny_inputs_variants(variant, precision):
    from paper_1905_03344_amd import ffi
    kw = {"grad_h": True} if variant == "grad_h" else {"gradients": ffi.SPH_GRADIENTS_IAD}
    kw["precision"] = ffi.SPH_FP64 if precision == "fp64" else ffi.SPH_MIXED
    print(f"tiny inputs {variant} {precision}", flush=True)
    ic0 = inputs.square_patch(4, 1).subset(np.array([], dtype=np.int64))
    sim0 = _sim(ic0, **kw)
    sim0.evaluate()
    sim0.sync()
    # one particle: no neighbours; Omega = 0 (its own term is the whole sum),
    # and its IAD moment matrix is zero, hence singular
    ic = inputs.square_patch(4, 1).subset(np.array([5]))
    sim = _sim(ic, **kw)
    sim.evaluate()
    if variant == "grad_h":
        code, stats = sim.sync()
        assert stats.nonconverged == 1
        assert abs(sim.omega()[0]) < 1e-15
        assert sim.numpy("ax")[0] == 0.0 and sim.numpy("du")[0] == 0.0
    else:
        with pytest.raises(ffi.SphError) as e:
            sim.sync()
        assert e.value.code == ffi.SPH_ENONFINITE


@pytest.mark.slow
def test_config2_full_size_parity():
    # 100^3 square patch, the launch configuration bench.py times
    ic = inputs.config_ic(2)
    print("config2 oracle ...", flush=True)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    print("config2 gpu ...", flush=True)
    sim = _sim(ic)
    sim.evaluate()
    sim.sync()
    compare_cells(sim, st)
    compare_neighbors(sim, st)
    compare_fields(sim, st)
