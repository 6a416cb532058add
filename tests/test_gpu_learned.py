"""GPU checks of the learned smoothing length: the bf16-MFMA MLP against
the oracle's bf16-emulating FP64 MLP, Adam, the feature build and harvest,
and the learned step against the plain step and the oracle.

MLP tolerances.  The two sides round the same operands to bfloat16, but the
GPU sums in FP32 and takes tanh in FP32, so a hidden activation that lies
within ~1e-6 of a bfloat16 rounding midpoint may round the other way (a
"flip", one bfloat16 ulp).  Each layer is therefore checked on the GPU's own
rounded inputs: its output must be the correctly rounded value or, near a
midpoint, the neighbouring one.  The output layer is checked to FP32
summation accuracy, and gradients normwise to 1e-3 per tensor."""
import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    return torch


def _bf16_bits_to_f64(bits):
    b = np.asarray(bits).astype(np.uint32) << np.uint32(16)
    return b.view(np.float32).astype(np.float64)


def _half_ulp_bf16(a):
    a = np.abs(np.asarray(a, dtype=np.float64))
    e = np.floor(np.log2(np.maximum(a, 1e-30)))
    return np.ldexp(1.0, (e - 8).astype(int))


def _check_rounded(gpu_bits, exact, slack=4e-6, max_flip_frac=0.01):
    """gpu value is bf16(exact) or, within `slack` of a midpoint, a neighbour."""
    g = _bf16_bits_to_f64(gpu_bits)
    r = O.bf16_round(exact)
    err = np.abs(g - exact)
    ok = (g == r) | (err <= _half_ulp_bf16(exact) + slack)
    assert np.all(ok), (np.max(err - _half_ulp_bf16(exact)), int(np.sum(~ok)))
    flips = np.mean(g != r)
    assert flips <= max_flip_frac, flips
    return flips


def _weights(seed, bias_scale=0.1):
    w = inputs.mlp_init(seed)
    u = inputs._stream(seed, 70, 129)
    w["b1"] = ((2 * u[:64] - 1) * bias_scale).astype(np.float32)
    w["b2"] = ((2 * u[64:128] - 1) * bias_scale).astype(np.float32)
    w["b3"] = np.array([(2 * u[128] - 1) * bias_scale], dtype=np.float32)
    return w


def _norm(seed):
    u = inputs._stream(seed, 71, 12)
    mean = (2 * u[:6] - 1) * 0.5
    std = 0.5 + u[6:]
    return np.concatenate([mean, std])


def _features(seed, n, norm):
    """raw FP32 rows whose standardised values spread over about [-2, 2]"""
    z, t = inputs.mlp_batch(seed, n, scale=2.0)
    raw = (z * norm[6:] + norm[:6]).astype(np.float32)
    rows = np.zeros((n, 8), dtype=np.float32)
    rows[:, :6] = raw
    return rows, t.astype(np.float32)


def _standardise(rows, norm):
    return (rows[:, :6].astype(np.float64) - norm[:6]) / norm[6:]


class MlpBox:
    """A bound context (tiny particle set) to run the MLP entry points on."""

    def __init__(self):
        from paper_1905_03344_amd.state import Simulation
        self.sim = Simulation(inputs.square_patch(4, 1))

    def set(self, w, norm):
        self.sim.set_mlp(w, norm)

    def dev(self, a):
        torch = _torch()
        return torch.from_numpy(np.ascontiguousarray(a)).to(self.sim.device)

    def forward(self, rows):
        torch = _torch()
        from paper_1905_03344_amd import ffi
        n = rows.shape[0]
        f = self.dev(rows)
        y = torch.zeros(max(n, 1), dtype=torch.float32, device=f.device)
        h1 = torch.zeros((max(n, 1), 64), dtype=torch.int16, device=f.device)
        h2 = torch.zeros((max(n, 1), 64), dtype=torch.int16, device=f.device)
        ffi.sph_mlp_forward(self.sim.ctx, f.data_ptr(), n, y.data_ptr(), h1.data_ptr(),
                            h2.data_ptr())
        return (y[:n].cpu().numpy().astype(np.float64),
                h1[:n].cpu().numpy().view(np.uint16), h2[:n].cpu().numpy().view(np.uint16))

    def backward(self, rows, target, order=None, row0=0, n=None):
        torch = _torch()
        from paper_1905_03344_amd import ffi
        n = rows.shape[0] if n is None else n
        f, t = self.dev(rows), self.dev(target)
        o = self.dev(order.astype(np.int32)) if order is not None else None
        g = torch.zeros(ffi.SPH_MLP_NPARAM + 1, dtype=torch.float32, device=f.device)
        ffi.sph_mlp_backward(self.sim.ctx, f.data_ptr(), t.data_ptr(),
                             o.data_ptr() if o is not None else None, row0, n, g.data_ptr())
        return g.cpu().numpy().astype(np.float64)


@pytest.fixture(scope="module")
def box():
    return MlpBox()


def _w64(w):
    return {k: np.asarray(v, dtype=np.float64) for k, v in w.items()}


@pytest.mark.parametrize("n", [1, 16, 1000, 4099])
def test_mlp_forward_layers(box, n):
    w, norm = _weights(11), _norm(12)
    box.set(w, norm)
    rows, _ = _features(13, n, norm)
    print(f"mlp forward n={n}", flush=True)
    y, h1, h2 = box.forward(rows)
    z = O.bf16_round(_standardise(rows, norm))
    W = {k: O.bf16_round(v) for k, v in _w64(w).items()}
    b1, b2, b3 = (np.asarray(w[k], dtype=np.float64) for k in ("b1", "b2", "b3"))
    a1 = np.tanh(z @ W["W1"].T + b1)
    _check_rounded(h1, a1)
    a2 = np.tanh(_bf16_bits_to_f64(h1) @ W["W2"].T + b2)
    _check_rounded(h2, a2)
    h2v = _bf16_bits_to_f64(h2)
    y_ref = h2v @ W["W3"].reshape(-1) + b3[0]
    cond = np.abs(h2v) @ np.abs(W["W3"].reshape(-1)) + abs(b3[0])
    assert np.all(np.abs(y - y_ref) <= 2e-6 * cond), np.max(np.abs(y - y_ref) / cond)
    # end to end against the oracle (flips allowed to move y slightly)
    *_, y_or = O.mlp_forward(_standardise(rows, norm), _w64(w), use_bf16=True)
    assert np.max(np.abs(y - y_or)) <= 1e-2 * max(np.max(np.abs(y_or)), 1e-3)
    assert np.median(np.abs(y - y_or)) <= 1e-5 * max(np.max(np.abs(y_or)), 1e-3)


def test_mlp_forward_empty(box):
    box.set(_weights(11), _norm(12))
    y, h1, h2 = box.forward(np.zeros((0, 8), dtype=np.float32))
    assert y.size == 0


def _grad_dict(g):
    from paper_1905_03344_amd.learned import unpack_params
    return unpack_params(g[:-1].astype(np.float32)), float(g[-1])


@pytest.mark.parametrize("n", [1, 37, 1000, 8192])
def test_mlp_backward_vs_oracle(box, n):
    w, norm = _weights(21), _norm(22)
    box.set(w, norm)
    rows, t = _features(23, n, norm)
    print(f"mlp backward n={n}", flush=True)
    g = box.backward(rows, t)
    gd, loss = _grad_dict(g)
    loss_or, g_or = O.mlp_loss_grad(_standardise(rows, norm), t, _w64(w), use_bf16=True)
    assert abs(loss - loss_or) <= 1e-4 * loss_or
    for k in g_or:
        ref = g_or[k].reshape(-1)
        got = gd[k].reshape(-1).astype(np.float64)
        scale = max(np.max(np.abs(ref)), 1e-30)
        assert np.max(np.abs(got - ref)) <= 1e-3 * scale, (k, np.max(np.abs(got - ref)) / scale)


def test_mlp_backward_rows_and_offset(box):
    """batch rows through an index list and a start offset"""
    w, norm = _weights(31), _norm(32)
    box.set(w, norm)
    rows, t = _features(33, 3000, norm)
    order = inputs.shuffle_order(34, 3000)
    g = box.backward(rows, t, order=order, row0=700, n=1100)
    sel = order[700:1800]
    loss_or, g_or = O.mlp_loss_grad(_standardise(rows[sel], norm), t[sel], _w64(w))
    gd, loss = _grad_dict(g)
    assert abs(loss - loss_or) <= 1e-4 * loss_or
    for k in g_or:
        ref = g_or[k].reshape(-1)
        got = gd[k].reshape(-1)
        assert np.max(np.abs(got - ref)) <= 1e-3 * max(np.max(np.abs(ref)), 1e-30), k
    # contiguous rows with an offset
    g2 = box.backward(rows, t, row0=1234, n=500)
    loss_or2, _ = O.mlp_loss_grad(_standardise(rows[1234:1734], norm), t[1234:1734], _w64(w))
    assert abs(g2[-1] - loss_or2) <= 1e-4 * loss_or2


def test_mlp_backward_deterministic(box):
    w, norm = _weights(41), _norm(42)
    box.set(w, norm)
    rows, t = _features(43, 5000, norm)
    a = box.backward(rows, t)
    b = box.backward(rows, t)
    np.testing.assert_array_equal(a, b)


def test_mlp_adam_vs_oracle(box):
    torch = _torch()
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.learned import pack_params
    w, norm = _weights(51), _norm(52)
    box.set(w, norm)
    p = pack_params(w).astype(np.float64)
    m = np.zeros_like(p)
    v = np.zeros_like(p)
    for t in (1, 2, 3):
        g = (2 * inputs._stream(53 + t, 72, p.size) - 1) * 0.05
        g32 = g.astype(np.float32)
        dg = torch.from_numpy(np.concatenate([g32, [0.0]]).astype(np.float32)).to(box.sim.device)
        ffi.sph_mlp_adam_step(box.sim.ctx, dg.data_ptr(), 1e-3, 0.9, 0.999, 1e-8, t)
        p, m, v = O.adam(p, m, v, g32.astype(np.float64), 1e-3, 0.9, 0.999, 1e-8, t)
        got, _ = box.sim.get_mlp()
        err = np.abs(got.astype(np.float64) - p)
        assert np.all(err <= 2e-7 * np.maximum(np.abs(p), 1.0) + 1e-9), np.max(err)
    # the bf16 copy follows the master weights: the forward sees RNE(master)
    master, _ = box.sim.get_mlp()
    from paper_1905_03344_amd.learned import unpack_params
    wm = unpack_params(master)
    rows, _ = _features(57, 200, norm)
    y, h1, h2 = box.forward(rows)
    W3 = O.bf16_round(np.asarray(wm["W3"], dtype=np.float64)).reshape(-1)
    y_ref = _bf16_bits_to_f64(h2) @ W3 + float(wm["b3"][0])
    cond = np.abs(_bf16_bits_to_f64(h2)) @ np.abs(W3) + abs(float(wm["b3"][0]))
    assert np.all(np.abs(y - y_ref) <= 2e-6 * cond)


def test_mlp_fit_norm(box):
    torch = _torch()
    from paper_1905_03344_amd import ffi
    box.set(_weights(61), None)
    rows = np.zeros((12345, 8), dtype=np.float32)
    rows[:, :6] = (inputs.gaussian(62, 73, 12345 * 6).reshape(-1, 6) * [1, 2, 3, 0.5, 0.1, 7]
                   + [0, 1, -2, 3, 0.2, -1]).astype(np.float32)
    rows[:, 3] = 0.25   # a constant feature: std 0 -> 1
    f = torch.from_numpy(rows).to(box.sim.device)
    ffi.sph_mlp_fit_norm(box.sim.ctx, f.data_ptr(), rows.shape[0])
    _, norm = box.sim.get_mlp()
    x = rows[:, :6].astype(np.float64)
    mean = x.mean(axis=0)
    std = x.std(axis=0)
    std[3] = 1.0
    np.testing.assert_allclose(norm[:6], mean, rtol=1e-12, atol=1e-14)
    np.testing.assert_allclose(norm[6:], std, rtol=1e-12)


def test_mlp_errors(box):
    from paper_1905_03344_amd import ffi
    with pytest.raises(ffi.SphError):
        box.sim.set_mlp(_weights(1), np.concatenate([np.zeros(6), np.zeros(6)]))
    with pytest.raises(ffi.SphError):
        ffi.sph_set_harvest(box.sim.ctx, 1, None)


# ---------------------------------------------------------------------------
# feature build and harvest
# ---------------------------------------------------------------------------

def _features_np(h, nc, rho, divv, m, pv, pu, gamma, dt):
    c = np.sqrt(gamma * (gamma - 1.0) * pu)
    vv = np.sqrt(pv[0] ** 2 + pv[1] ** 2 + pv[2] ** 2)
    return np.stack([np.log(h), nc / 100.0 - 1.0, np.log(rho * h ** 3 / m), dt * divv,
                     dt * vv / h, dt * c / h], axis=1)


def test_features_and_harvest():
    torch = _torch()
    from paper_1905_03344_amd.state import Simulation
    ic = inputs.square_patch(18, 5)
    sim = Simulation(ic)
    sim.evaluate()
    sim.step(0.0)
    sim.sync()
    # standalone feature rows of the current state at the device dt
    feat = sim.features().cpu().numpy()
    g = sim.params.gamma
    ref = _features_np(sim.numpy("h"), sim.numpy("nc"), sim.numpy("rho"), sim.numpy("divv"),
                       sim.numpy("m"), (sim.numpy("pvx"), sim.numpy("pvy"), sim.numpy("pvz")),
                       sim.numpy("pu"), g, sim.dt())
    np.testing.assert_allclose(feat[:, :6], ref.astype(np.float32), rtol=3e-7, atol=1e-30)
    assert np.all(feat[:, 6:] == 0)
    # harvest across one step: rows in the order of that step
    before = {k: sim.numpy(k).copy() for k in ("h", "nc", "rho", "divv", "m")}
    dt = sim.dt()
    F = torch.zeros((ic.n, 8), dtype=torch.float32, device=sim.device)
    T = torch.zeros(ic.n, dtype=torch.float32, device=sim.device)
    sim.set_harvest(F, T)
    sim.step(0.0)
    sim.set_harvest(None, None)
    sim.sync()
    perm = sim.numpy("perm")
    F = F.cpu().numpy()
    T = T.cpu().numpy()
    b = {k: v[perm] for k, v in before.items()}
    np.testing.assert_allclose(F[:, 0], np.log(b["h"]).astype(np.float32), rtol=3e-7)
    np.testing.assert_allclose(F[:, 1], (b["nc"] / 100.0 - 1.0).astype(np.float32), rtol=3e-7,
                               atol=1e-8)
    np.testing.assert_allclose(F[:, 2], np.log(b["rho"] * b["h"] ** 3 / b["m"]).astype(np.float32),
                               rtol=3e-7, atol=1e-7)
    np.testing.assert_allclose(F[:, 3], (dt * b["divv"]).astype(np.float32), rtol=3e-7, atol=1e-12)
    pv = (sim.numpy("pvx"), sim.numpy("pvy"), sim.numpy("pvz"))
    np.testing.assert_allclose(F[:, 4], (dt * np.sqrt(sum(a * a for a in pv)) / b["h"]).astype(np.float32),
                               rtol=3e-7, atol=1e-12)
    c = np.sqrt(g * (g - 1.0) * sim.numpy("pu"))
    np.testing.assert_allclose(F[:, 5], (dt * c / b["h"]).astype(np.float32), rtol=3e-7, atol=1e-12)
    # solved target: log(h_new) - f1
    ys = np.log(sim.numpy("h")) - F[:, 0].astype(np.float64)
    np.testing.assert_allclose(T, ys.astype(np.float32), rtol=1e-6, atol=1e-7)
    # centred target: log(h_new (100 / N_new)^(1/3)) - f1, on the next step
    from paper_1905_03344_amd import ffi
    F2 = torch.zeros((ic.n, 8), dtype=torch.float32, device=sim.device)
    T2 = torch.zeros(ic.n, dtype=torch.float32, device=sim.device)
    sim.set_harvest(F2, T2, ffi.SPH_TARGET_CENTRED)
    sim.step(0.0)
    sim.set_harvest(None, None)
    sim.sync()
    F2 = F2.cpu().numpy()
    yc = (np.log(sim.numpy("h")) - F2[:, 0].astype(np.float64)
          + np.log(100.0 / sim.numpy("nc")) / 3.0)
    np.testing.assert_allclose(T2.cpu().numpy(), yc.astype(np.float32), rtol=1e-6, atol=1e-7)


# ---------------------------------------------------------------------------
# learned step
# ---------------------------------------------------------------------------

FIELDS = ("x", "y", "z", "vx", "vy", "vz", "h", "u", "nc", "rho", "divv", "ax", "ay", "az", "du")


def _run(ic, h_mode, w=None, norm=None, steps=2, **kw):
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(ic, h_mode=h_mode, **kw)
    if w is not None:
        sim.set_mlp(w, norm)
    sim.evaluate()
    stats = []
    for _ in range(steps):
        sim.step(0.0)
        stats.append(sim.sync()[1])
    return sim, stats


def test_learned_zero_last_layer_is_plain():
    from paper_1905_03344_amd import ffi
    ic = inputs.square_patch(20, inputs.CONFIG_SEEDS[1])
    w = _weights(81)
    w["W3"][:] = 0
    w["b3"][:] = 0
    plain, _ = _run(ic, ffi.SPH_H_PLAIN)
    learn, st = _run(ic, ffi.SPH_H_LEARNED, w, _norm(82))
    for f in FIELDS:
        np.testing.assert_array_equal(plain.numpy(f), learn.numpy(f), err_msg=f)
    for s in st:
        assert s.learned_accepted + s.learned_fallback == ic.n
        assert s.learned_accepted > 0


def test_learned_forced_fallback_is_plain():
    from paper_1905_03344_amd import ffi
    ic = inputs.square_patch(20, inputs.CONFIG_SEEDS[1])
    w = _weights(83)
    w["b3"][:] = 50.0   # y clamps at 1/2: h_try = 1.65 h, counts ~4.5x the target
    plain, _ = _run(ic, ffi.SPH_H_PLAIN)
    learn, st = _run(ic, ffi.SPH_H_LEARNED, w, _norm(84))
    for f in FIELDS:
        np.testing.assert_array_equal(plain.numpy(f), learn.numpy(f), err_msg=f)
    for s in st:
        assert s.learned_fallback == ic.n and s.learned_accepted == 0
    assert not np.any(learn.numpy("flags") & ffi.SPH_FLAG_LEARNED)


def test_learned_requires_weights():
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(inputs.square_patch(6, 1), h_mode=ffi.SPH_H_LEARNED)
    sim.evaluate()
    with pytest.raises(ffi.SphError):
        sim.step(0.0)


@pytest.fixture(scope="module")
def trained_small():
    """A model trained on 10 plain steps of a 20^3 patch (seed A)."""
    from paper_1905_03344_amd import learned
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(inputs.square_patch(20, 101))
    sim.evaluate()
    feat, target = learned.harvest(sim, steps=10)
    sim.sync()
    w, norm, losses = learned.train(sim, feat, target, seed=102, epochs=4, batch=1024)
    return w, norm, losses


def test_training_reduces_loss(trained_small):
    w, norm, losses = trained_small
    assert np.all(np.isfinite(losses))
    k = max(len(losses) // 8, 1)
    assert np.mean(losses[-k:]) < 0.5 * np.mean(losses[:k]), (losses[:k], losses[-k:])


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_learned_step_vs_oracle(trained_small, precision):
    """Learned step on another seed: cells and lists exact, accepted h in
    band with the oracle's exact count, fallback h identical to the plain
    iteration's, fields at the learned form's own h against the oracle."""
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation
    from test_gpu_parity import _upload_oracle_state, compare_cells, compare_neighbors, compare_fields
    w, norm, _ = trained_small
    ic = inputs.square_patch(20, 202)
    st = O.State(ic.copy())
    st.keep_gather = True
    st.evaluate(method=1)
    prec = ffi.SPH_FP64 if precision == "fp64" else ffi.SPH_MIXED
    sim = Simulation(ic, h_mode=ffi.SPH_H_LEARNED, precision=prec)
    sim.set_mlp(w, norm)
    _upload_oracle_state(sim, st)
    # the Courant dt, as in the steps the model was trained on (the
    # features f4..f6 scale with dt)
    dt = st.dt_next
    plain = O.State(ic.copy())
    plain.f = {k: v.copy() for k, v in st.f.items()}
    plain.step(dt, method=1)
    sim.step(dt)
    code, stats = sim.sync()
    h = sim.numpy("h")
    flags = sim.numpy("flags")
    acc = (flags & ffi.SPH_FLAG_LEARNED) != 0
    print(f"learned {precision}: accepted {acc.mean():.3f}", flush=True)
    assert stats.learned_accepted == int(acc.sum())
    assert stats.learned_accepted + stats.learned_fallback == ic.n
    assert acc.any()
    # fallback particles: exactly the plain iteration's h
    np.testing.assert_array_equal(h[~acc], plain.f["h"][~acc])
    # the oracle at the GPU's h
    st.h_given = h
    st.step(dt, method=1)
    compare_cells(sim, st)
    np.testing.assert_array_equal(sim.numpy("nc"), st.f["nc"])
    assert np.all(np.abs(st.f["nc"][acc] - 100) <= 5)
    compare_neighbors(sim, st)
    if precision == "fp64":
        compare_fields(sim, st)
    else:
        from test_gpu_mixed import check_mixed_fields
        check_mixed_fields(sim, st)


def test_learned_try_shell_speed_only(trained_small):
    """The learned try's shell (never, always, chosen per solve) changes only
    how the misses are counted: fields, h, counts, flags and the
    accepted/fallback split are the same bit for bit over three steps of a
    patch on which many tries miss (AUTO records none at this size)."""
    from paper_1905_03344_amd import ffi
    w, norm, _ = trained_small
    ic = inputs.square_patch(20, 202)
    modes = (ffi.SPH_TRY_SHELL_NEVER, ffi.SPH_TRY_SHELL_ALWAYS, ffi.SPH_TRY_SHELL_AUTO)
    runs = {m: _run(ic, ffi.SPH_H_LEARNED, w, norm, steps=3, learned_try_shell=m) for m in modes}
    ref, rst = runs[ffi.SPH_TRY_SHELL_NEVER]
    for m in modes[1:]:
        sim, st = runs[m]
        for f in FIELDS + ("flags",):
            np.testing.assert_array_equal(ref.numpy(f), sim.numpy(f), err_msg=f"mode {m}: {f}")
        for a, b in zip(rst, st):
            assert (a.learned_accepted, a.learned_fallback) == (b.learned_accepted,
                                                                 b.learned_fallback)
    miss = [s.learned_fallback / ic.n for s in rst]
    cand = {m: [s.candidates for s in runs[m][1]] for m in modes}
    counts = {m: [s.h_counts for s in runs[m][1]] for m in modes}
    print(f"misses {miss}; candidates {cand}; counts {counts}", flush=True)
    assert min(miss) > 0.1   # many misses: the shell saves walks
    assert sum(cand[ffi.SPH_TRY_SHELL_ALWAYS]) < sum(cand[ffi.SPH_TRY_SHELL_NEVER])
