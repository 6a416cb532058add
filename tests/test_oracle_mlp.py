"""Pins for the oracle's learned smoothing-length MLP: bf16 rounding against
an exact rational rounding and against torch's float32->bfloat16 conversion,
analytic gradients against central finite differences, Adam against its
closed form on the first step."""
import math
from fractions import Fraction

import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs


def _round_sig8(v):
    # exact rational round-to-nearest-even to 8 significant bits
    if v == 0 or not math.isfinite(v):
        return v
    m, e = math.frexp(abs(v))        # v = m 2^e, m in [0.5, 1)
    q = Fraction(abs(v)) / Fraction(2) ** (e - 8)   # in [128, 256)
    fl = math.floor(q)
    rem = q - fl
    if rem > Fraction(1, 2) or (rem == Fraction(1, 2) and fl % 2 == 1):
        fl += 1
    return math.copysign(float(Fraction(fl) * Fraction(2) ** (e - 8)), v)


def test_bf16_round_exact_rational():
    rng = np.random.default_rng(5)
    v = np.concatenate([rng.standard_normal(2000) * 10.0 ** rng.integers(-6, 6, 2000),
                        [1.0 + 2.0 ** -8, 1.0 + 3 * 2.0 ** -8, -(1.0 + 2.0 ** -8) , 255.5, 0.0]])
    out = O.bf16_round(v)
    np.testing.assert_array_equal(out, [_round_sig8(float(a)) for a in v])


def test_bf16_round_matches_torch_on_floats():
    torch = pytest.importorskip("torch")
    rng = np.random.default_rng(6)
    f = (rng.standard_normal(5000) * 3).astype(np.float32)
    ref = torch.from_numpy(f).to(torch.bfloat16).to(torch.float64).numpy()
    np.testing.assert_array_equal(O.bf16_round(f.astype(np.float64)), ref)


def test_forward_shapes_and_tanh_range():
    w = inputs.mlp_init(7)
    x, t = inputs.mlp_batch(3, 64)
    z1, a1, z2, a2, y = O.mlp_forward(x, w)
    assert y.shape == (64,) and np.all(np.abs(a1) <= 1) and np.all(np.abs(a2) <= 1)
    np.testing.assert_allclose(np.tanh(z1), a1, rtol=1e-15)
    # a zeroed last layer returns the bias exactly
    w0 = dict(w)
    w0["W3"] = np.zeros_like(w["W3"])
    w0["b3"] = np.array([0.25], dtype=np.float32)
    assert np.all(O.mlp_forward(x, w0)[4] == 0.25)


def test_gradients_finite_difference():
    w = {k: v.astype(np.float64) for k, v in inputs.mlp_init(11).items()}
    for k in w:
        if k.startswith("b"):
            w[k] = w[k] + 0.05 * np.arange(w[k].size).reshape(w[k].shape) / w[k].size
    x, t = inputs.mlp_batch(12, 16)
    loss, g = O.mlp_loss_grad(x, t, w, use_bf16=False)
    rng = np.random.default_rng(0)
    for k in ("W1", "b1", "W2", "b2", "W3", "b3"):
        flat = w[k].ravel()
        for e in rng.choice(flat.size, size=min(8, flat.size), replace=False):
            eps = 1e-6
            wp = {kk: vv.copy() for kk, vv in w.items()}
            wm = {kk: vv.copy() for kk, vv in w.items()}
            wp[k].ravel()[e] += eps
            wm[k].ravel()[e] -= eps
            lp = np.mean((O.mlp_forward(x, wp, use_bf16=False)[4] - t) ** 2)
            lm = np.mean((O.mlp_forward(x, wm, use_bf16=False)[4] - t) ** 2)
            fd = (lp - lm) / (2 * eps)
            assert abs(fd - g[k].ravel()[e]) < 1e-7 * max(1.0, abs(fd)), (k, e, fd, g[k].ravel()[e])
    assert loss == pytest.approx(np.mean((O.mlp_forward(x, w, use_bf16=False)[4] - t) ** 2),
                                 rel=1e-13)


def test_bf16_loss_close_to_fp64_loss():
    w = inputs.mlp_init(2)
    x, t = inputs.mlp_batch(4, 256)
    l16, g16 = O.mlp_loss_grad(x, t, w, use_bf16=True)
    l64, g64 = O.mlp_loss_grad(x, t, w, use_bf16=False)
    assert abs(l16 - l64) < 0.02 * l64
    for k in g16:
        assert np.linalg.norm(g16[k] - g64[k]) < 0.05 * (np.linalg.norm(g64[k]) + 1e-12)


def test_adam_first_step_closed_form():
    rng = np.random.default_rng(1)
    p = rng.standard_normal(10); g = rng.standard_normal(10)
    p1, m1, v1 = O.adam(p, np.zeros(10), np.zeros(10), g, lr=1e-3, t=1)
    # at t = 1 the bias-corrected moments are g and g^2: step = lr * sign-ish
    np.testing.assert_allclose(p1, p - 1e-3 * g / (np.abs(g) + 1e-8), rtol=1e-12)
    np.testing.assert_allclose(m1, 0.1 * g, rtol=1e-15)
    np.testing.assert_allclose(v1, 0.001 * g * g, rtol=1e-12)


def test_training_reduces_loss():
    w = {k: v.astype(np.float64) for k, v in inputs.mlp_init(5).items()}
    x, _ = inputs.mlp_batch(6, 512)
    t = 0.3 * np.tanh(x[:, 0] - 0.5 * x[:, 2])     # a learnable target
    state = {k: (np.zeros_like(v), np.zeros_like(v)) for k, v in w.items()}
    l0 = None
    for it in range(1, 201):
        loss, g = O.mlp_loss_grad(x, t, w, use_bf16=True)
        l0 = loss if l0 is None else l0
        for k in w:
            w[k], m, v = O.adam(w[k], *state[k], g[k], lr=3e-3, t=it)
            state[k] = (m, v)
    assert loss < 0.1 * l0
