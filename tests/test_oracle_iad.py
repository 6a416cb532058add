"""Pins for the oracle's IAD (integral approach to derivatives) matrices and
IAD momentum and energy equations: the inverse of a brute-force moment sum,
exact gradients of linear fields, closed forms on a cubic lattice under
linear pressure and velocity fields, the assembly with one pressurised
particle, antisymmetry and conservation."""
import math

import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs


def _m4(r, h):
    q = r / h
    w = np.where(q < 1.0, 1.0 - 1.5 * q * q + 0.75 * q ** 3,
                 np.where(q < 2.0, 0.25 * (2.0 - q) ** 3, 0.0))
    return w / (math.pi * h ** 3)


def _all_pairs(n):
    off = np.arange(n + 1, dtype=np.int64) * (n - 1)
    idx = np.array([j for i in range(n) for j in range(n) if j != i], dtype=np.int32)
    return off, idx


def _cloud(seed=3, side=5):
    g = np.arange(side, dtype=float)
    x, y, z = (a.ravel() for a in np.meshgrid(g, g, g, indexing="ij"))
    rng = np.random.default_rng(seed)
    pos = np.stack([x, y, z], 1) + 0.25 * rng.standard_normal((side ** 3, 3))
    n = side ** 3
    m = 1.0 + 0.3 * rng.random(n)
    h = 1.2 + 0.4 * rng.random(n)
    rho = 0.8 + 0.5 * rng.random(n)
    return pos, m, h, rho


def _unpack(c6):
    c = np.empty((len(c6), 3, 3))
    c[:, 0, 0], c[:, 0, 1], c[:, 0, 2] = c6[:, 0], c6[:, 1], c6[:, 2]
    c[:, 1, 0], c[:, 1, 1], c[:, 1, 2] = c6[:, 1], c6[:, 3], c6[:, 4]
    c[:, 2, 0], c[:, 2, 1], c[:, 2, 2] = c6[:, 2], c6[:, 4], c6[:, 5]
    return c


def test_iad_matrix_inverts_moments_and_differentiates_linear_fields():
    pos, m, h, rho = _cloud()
    n = len(m)
    off, idx = _all_pairs(n)
    c6, bad = O.iad_matrices(*pos.T, m, rho, h, (0, 0, 0), (0, 0, 0), (0, 0, 0), off, idx)
    assert bad == 0
    c = _unpack(c6)
    d = pos[None, :, :] - pos[:, None, :]              # d[i, j] = x_j - x_i
    r = np.sqrt(np.sum(d * d, axis=2))
    W = _m4(r, h[:, None])                             # W(r_ij, h_i), zero beyond 2 h_i
    V = m / rho
    tau = np.einsum("j,ij,ija,ijb->iab", V, W, d, d)
    eye = np.einsum("iab,ibc->iac", c, tau)
    np.testing.assert_allclose(eye, np.broadcast_to(np.eye(3), eye.shape), atol=1e-12)
    # the estimator sum_j V_j (f_j - f_i) c_i d W is exact for f = a + b.x
    rng = np.random.default_rng(1)
    for _ in range(3):
        a0, b = rng.standard_normal(), rng.standard_normal(3)
        f = a0 + pos @ b
        A = np.einsum("iab,ijb->ija", c, d) * W[:, :, None]
        grad = np.einsum("j,ij,ija->ia", V, f[None, :] - f[:, None], A)
        np.testing.assert_allclose(grad, np.broadcast_to(b, grad.shape), rtol=0, atol=1e-11)


def test_iad_singular_matrix_reported():
    # particles on one line: every moment matrix is rank one
    n = 6
    x = np.arange(n, dtype=float) * 0.5
    z = np.zeros(n)
    off, idx = _all_pairs(n)
    c6, bad = O.iad_matrices(x, z, z, np.ones(n), np.ones(n), np.full(n, 1.0), (0, 0, 0),
                             (0, 0, 0), (0, 0, 0), off, idx)
    assert bad == n and np.all(np.isnan(c6))


def _interior_lattice(n_side=16, h_over_s=1.5):
    ps = inputs.perfect_lattice(n_side, h_over_s, periodic_all=False)
    off, idx = O.lists(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo, ps.box_hi)
    rho, _ = O.density(ps.x, ps.y, ps.z, ps.vx, ps.vy, ps.vz, ps.m, ps.h, ps.periodic,
                       ps.box_lo, ps.box_hi, off, idx)
    c6, bad = O.iad_matrices(ps.x, ps.y, ps.z, ps.m, rho, ps.h, ps.periodic, ps.box_lo,
                             ps.box_hi, off, idx)
    assert bad == 0
    # particles whose neighbours' neighbourhoods are complete lattice shells
    s = ps.meta["s"]
    margin = 4.0 * ps.h[0] + s
    pos = np.stack([ps.x, ps.y, ps.z], 1)
    inner = np.all((pos > margin) & (pos < 1.0 - margin), axis=1)
    assert inner.sum() >= 8
    return ps, off, idx, rho, c6, inner


def test_iad_lattice_linear_pressure_exact_gradient():
    ps, off, idx, rho, c6, inner = _interior_lattice()
    g = np.array([0.3, -1.1, 0.7])
    P = 2.0 + ps.x * g[0] + ps.y * g[1] + ps.z * g[2]
    c = np.ones(ps.n)
    args = (ps.x, ps.y, ps.z, ps.vx, ps.vy, ps.vz, ps.m, ps.h, rho, P, c, ps.periodic,
            ps.box_lo, ps.box_hi, off, idx)
    ax, ay, az, *_ = O.forces(*args, alpha=0.0, beta=0.0, iad=c6)
    r0 = rho[inner][0]
    np.testing.assert_allclose(rho[inner], r0, rtol=1e-14)
    for a, gd in zip((ax, ay, az), g):
        np.testing.assert_allclose(a[inner], -gd / r0, rtol=1e-10)
    # the kernel-derivative form is only approximately -grad P / rho here
    kx, *_ = O.forces(*args, alpha=0.0, beta=0.0)
    assert np.max(np.abs(kx[inner] + g[0] / r0)) > 1e-6 * abs(g[0] / r0)


def test_iad_lattice_linear_velocity_first_law():
    ps, off, idx, rho, c6, inner = _interior_lattice()
    L = np.array([[0.2, -0.5, 0.1], [0.4, -0.3, 0.25], [-0.15, 0.35, 0.6]])
    pos = np.stack([ps.x, ps.y, ps.z], 1)
    v = pos @ L.T
    P = np.full(ps.n, 1.7)
    c = np.ones(ps.n)
    ax, ay, az, du, *_ = O.forces(ps.x, ps.y, ps.z, *v.T, ps.m, ps.h, rho, P, c, ps.periodic,
                                  ps.box_lo, ps.box_hi, off, idx, alpha=0.0, beta=0.0, iad=c6)
    r0 = rho[inner][0]
    # du/dt = -(P / rho) div v, and no net force under uniform pressure
    np.testing.assert_allclose(du[inner], -1.7 / r0 * np.trace(L), rtol=1e-10)
    assert np.max(np.abs(np.concatenate([ax[inner], ay[inner], az[inner]]))) < 1e-10


def test_iad_single_pressurised_particle_assembly():
    pos, m, h, rho = _cloud(seed=7)
    n = len(m)
    off, idx = _all_pairs(n)
    c6, bad = O.iad_matrices(*pos.T, m, rho, h, (0, 0, 0), (0, 0, 0), (0, 0, 0), off, idx)
    c = _unpack(c6)
    k = 62
    P = np.zeros(n)
    P[k] = 1.3
    vel = np.zeros_like(pos)
    ax, ay, az, du, *_ = O.forces(*pos.T, *vel.T, m, h, rho, P, np.ones(n), (0, 0, 0),
                                  (0, 0, 0), (0, 0, 0), off, idx, alpha=0.0, beta=0.0, iad=c6)
    a = np.stack([ax, ay, az], 1)
    pk = P[k] / rho[k] ** 2
    # particle k: its own matrix over its neighbours, d = x_j - x_k, W with h_k
    d = pos - pos[k]
    Wk = _m4(np.sqrt(np.sum(d * d, 1)), h[k])
    expect_k = -pk * c[k] @ np.sum(m[:, None] * d * Wk[:, None], 0)
    np.testing.assert_allclose(a[k], expect_k, rtol=1e-12)
    # a neighbour q feels k's pressure through k's matrix: -m_k pk c_k (x_k - x_q) W(r, h_k)
    for q in np.nonzero((Wk > 0) & (np.arange(n) != k))[0][:10]:
        expect_q = -m[k] * pk * c[k] @ (pos[k] - pos[q]) * Wk[q]
        np.testing.assert_allclose(a[q], expect_q, rtol=1e-12, atol=1e-14 * np.max(np.abs(a)))


def _patch(seed=4):
    ps = inputs.square_patch(12, seed)
    rng = np.random.default_rng(seed)
    ps.vx = ps.vx + 0.3 * rng.standard_normal(ps.n)
    ps.vy = ps.vy + 0.3 * rng.standard_normal(ps.n)
    ps.vz = ps.vz + 0.3 * rng.standard_normal(ps.n)
    ps.u = 1.0 + 0.2 * rng.random(ps.n)
    h, *_ = O.hsolve(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo, ps.box_hi)
    ps.h = h * (1.0 + 0.05 * rng.random(ps.n))
    ps.periodic = (0, 0, 0)
    off, idx = O.lists(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo, ps.box_hi)
    rho, _ = O.density(ps.x, ps.y, ps.z, ps.vx, ps.vy, ps.vz, ps.m, ps.h, ps.periodic,
                       ps.box_lo, ps.box_hi, off, idx)
    P, c = O.eos(rho, ps.u)
    c6, bad = O.iad_matrices(ps.x, ps.y, ps.z, ps.m, rho, ps.h, ps.periodic, ps.box_lo,
                             ps.box_hi, off, idx)
    assert bad == 0
    return ps, off, idx, rho, P, c, c6


def test_iad_pair_term_antisymmetric_and_conservative():
    ps, off, idx, rho, P, c, c6 = _patch()
    args = (ps.x, ps.y, ps.z, ps.vx, ps.vy, ps.vz, ps.m, ps.h, rho, P, c, ps.periodic,
            ps.box_lo, ps.box_hi)
    rng = np.random.default_rng(0)
    for i in rng.integers(0, ps.n, 40):
        for j in idx[off[i]:off[i + 1]][:12]:
            a = O.pair_term(*args, int(i), int(j), iad=c6)
            b = O.pair_term(*args, int(j), int(i), iad=c6)
            assert np.array_equal(a[:3], -b[:3]) and a[3] == b[3]
    ax, ay, az, du, dt_i, amag = O.forces(*args, off, idx, iad=c6)
    m = ps.m
    scale = np.sum(m * amag)
    for a in (ax, ay, az):
        assert abs(np.sum(m * a)) < 1e-13 * scale
    vmag = np.sqrt(ps.vx ** 2 + ps.vy ** 2 + ps.vz ** 2)
    dE = np.sum(m * (ps.vx * ax + ps.vy * ay + ps.vz * az + du))
    assert abs(dE) < 1e-12 * np.sum(m * amag * vmag)
    # differs from the kernel-derivative form on an irregular set
    kx, *_ = O.forces(*args, off, idx)
    assert np.max(np.abs(kx - ax)) > 1e-3 * np.max(np.abs(kx))


def test_state_iad_switch():
    ps = inputs.square_patch(8, 1)
    s0 = O.State(ps, O.Params())
    s1 = O.State(ps, O.Params(gradients=O.GRADIENTS_IAD))
    s0.evaluate()
    s1.evaluate()
    np.testing.assert_array_equal(s0.f["rho"], s1.f["rho"])
    assert s1.iad is not None and s1.iad.shape == (ps.n, 6)
    assert not np.array_equal(s0.f["ax"], s1.f["ax"])
