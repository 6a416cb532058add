"""Pins for the oracle's grad-h correction terms (the accuracy variant that
takes the smoothing length as a function of density, h = eta (m/rho)^(1/3)).

With h tied to rho that way and no viscosity, the momentum and energy
equations with the grad-h factors Omega are the exact derivatives of the
thermal energy E = sum_i m_i u_i(rho_i) of an adiabatic gas:
  m_i a_i = -dE/dr_i,   du_i/dt = (P_i / rho_i^2) d rho_i / dt.
The tests below solve the h-rho relation to convergence by brute force, take
those derivatives by central finite differences, and compare them with the
oracle's forces -- a check that does not pass through the oracle's formulas."""
import math

import numpy as np
import pytest

import oracle as O

ETA = 1.3
K_ADIA = 0.7
GAMMA = 5.0 / 3.0


def _m4(r, h):
    # the cubic spline (3-D normalisation 1/pi), vectorised; pinned against the
    # oracle's own kernel below
    q = r / h
    w = np.where(q < 1.0, 1.0 - 1.5 * q * q + 0.75 * q ** 3,
                 np.where(q < 2.0, 0.25 * (2.0 - q) ** 3, 0.0))
    return w / (math.pi * h ** 3)


def test_vector_m4_matches_oracle_kernel():
    for r in np.linspace(0.0, 2.3, 47):
        for h in (0.7, 1.0, 1.9):
            assert _m4(np.array(r), h) == pytest.approx(O.kernel_w(r, h), rel=1e-14, abs=1e-300)


@pytest.mark.parametrize("kernel", [O.KERNEL_M4, O.KERNEL_WENDLAND, O.KERNEL_SINC5])
def test_dwdh_is_derivative_in_h(kernel):
    wf = {O.KERNEL_M4: O.kernel_w, O.KERNEL_WENDLAND: O.kernel_wendland,
          O.KERNEL_SINC5: O.kernel_sinc}[kernel]
    for r in (0.0, 0.3, 0.99, 1.4, 1.9):
        h, e = 1.1, 1e-5
        fd = (wf(r, h + e) - wf(r, h - e)) / (2 * e)
        assert O.kernel_dwdh(r, h, kernel) == pytest.approx(fd, rel=2e-8, abs=1e-10)
    assert O.kernel_dwdh(2.5, 1.0, kernel) == 0.0


def _cloud(seed=3, side=5):
    g = np.arange(side, dtype=float)
    x, y, z = (a.ravel() for a in np.meshgrid(g, g, g, indexing="ij"))
    rng = np.random.default_rng(seed)
    pos = np.stack([x, y, z], 1) + 0.2 * rng.standard_normal((side ** 3, 3))
    m = 1.0 + 0.3 * rng.random(side ** 3)
    return pos, m


def _rho_of(pos, m, h):
    d = pos[:, None, :] - pos[None, :, :]
    r = np.sqrt(np.sum(d * d, axis=2))
    return np.sum(m[None, :] * _m4(r, h[:, None]), axis=1)


def _solve_h(pos, m, h0=None):
    # Newton on f(h) = h - eta (m / rho(h))^(1/3), per particle, with the
    # derivative of rho in h taken by a central difference
    h = np.full(len(m), 1.4) if h0 is None else h0.copy()
    for _ in range(60):
        rho = _rho_of(pos, m, h)
        e = 1e-6 * h
        drho = (_rho_of(pos, m, h + e) - _rho_of(pos, m, h - e)) / (2 * e)
        f = h - ETA * np.cbrt(m / rho)
        fp = 1.0 + ETA * np.cbrt(m) / 3.0 * rho ** (-4.0 / 3.0) * drho
        step = f / fp
        h = h - step
        if np.max(np.abs(step) / h) < 1e-15:
            break
    return h


def _energy(pos, m):
    h = _solve_h(pos, m)
    rho = _rho_of(pos, m, h)
    return np.sum(m * K_ADIA * rho ** (GAMMA - 1) / (GAMMA - 1))


def _all_pairs(n):
    off = np.arange(n + 1, dtype=np.int64) * (n - 1)
    idx = np.array([j for i in range(n) for j in range(n) if j != i], dtype=np.int32)
    return off, idx


def _oracle_fields(pos, m, vel, h):
    n = len(m)
    off, idx = _all_pairs(n)
    rho, divv, omega = O.density(*pos.T, *vel.T, m, h, (0, 0, 0), (0, 0, 0), (0, 0, 0),
                                 off, idx, with_omega=True)
    P = K_ADIA * rho ** GAMMA
    c = np.sqrt(GAMMA * P / rho)
    return off, idx, rho, P, c, omega


def test_omega_is_one_plus_log_derivative_of_rho():
    pos, m = _cloud()
    h = _solve_h(pos, m)
    vel = np.zeros_like(pos)
    off, idx, rho, P, c, omega = _oracle_fields(pos, m, vel, h)
    np.testing.assert_allclose(rho, _rho_of(pos, m, h), rtol=1e-13)
    e = 1e-5 * h
    dlnrho = (_rho_of(pos, m, h + e) - _rho_of(pos, m, h - e)) / (2 * e) * h / rho
    np.testing.assert_allclose(omega, 1.0 + dlnrho / 3.0, rtol=1e-8)
    # a non-trivial correction: the cloud's edge particles are far from 1
    assert np.max(np.abs(omega - 1.0)) > 0.05


def test_grad_h_force_is_energy_gradient():
    pos, m = _cloud()
    n = len(m)
    h = _solve_h(pos, m)
    vel = np.zeros_like(pos)
    off, idx, rho, P, c, omega = _oracle_fields(pos, m, vel, h)
    ax, ay, az, du, dt_i, amag = O.forces(*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0),
                                          (0, 0, 0), off, idx, alpha=0.0, beta=0.0,
                                          omega=omega)
    a = np.stack([ax, ay, az], 1)
    # the averaged-gradient form is not the energy gradient: it must differ
    bx, by, bz, *_ = O.forces(*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0), (0, 0, 0),
                              off, idx, alpha=0.0, beta=0.0)
    b = np.stack([bx, by, bz], 1)
    scale = np.max(np.abs(a))
    rng = np.random.default_rng(0)
    eps = 1e-5
    worst_gh, worst_avg = 0.0, 0.0
    for i in rng.choice(n, 12, replace=False):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += eps
            pm[i, d] -= eps
            g = -(_energy(pp, m) - _energy(pm, m)) / (2 * eps) / m[i]
            worst_gh = max(worst_gh, abs(a[i, d] - g))
            worst_avg = max(worst_avg, abs(b[i, d] - g))
    assert worst_gh < 1e-6 * scale
    assert worst_avg > 1e-3 * scale


def test_grad_h_energy_rate_is_adiabatic():
    pos, m = _cloud(seed=8)
    n = len(m)
    h = _solve_h(pos, m)
    rng = np.random.default_rng(5)
    vel = rng.standard_normal(pos.shape)
    off, idx, rho, P, c, omega = _oracle_fields(pos, m, vel, h)
    ax, ay, az, du, dt_i, amag = O.forces(*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0),
                                          (0, 0, 0), off, idx, alpha=0.0, beta=0.0,
                                          omega=omega)
    # d rho_i / dt along the flow, h re-solved at each displaced configuration
    eps = 1e-6
    rp = _rho_of(pos + eps * vel, m, _solve_h(pos + eps * vel, m, h))
    rm = _rho_of(pos - eps * vel, m, _solve_h(pos - eps * vel, m, h))
    expect = P / rho ** 2 * (rp - rm) / (2 * eps)
    np.testing.assert_allclose(du, expect, rtol=0, atol=1e-6 * np.max(np.abs(expect)))
    # and the total energy rate vanishes, to rounding
    dE = np.sum(m * (vel[:, 0] * ax + vel[:, 1] * ay + vel[:, 2] * az + du))
    vmag = np.sqrt(np.sum(vel * vel, 1))
    assert abs(dE) < 1e-12 * np.sum(m * amag * vmag)


def test_grad_h_pair_term_antisymmetric_with_viscosity():
    pos, m = _cloud(seed=2)
    h = _solve_h(pos, m)
    vel = np.random.default_rng(1).standard_normal(pos.shape)
    off, idx, rho, P, c, omega = _oracle_fields(pos, m, vel, h)
    args = (*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0), (0, 0, 0))
    for i, j in [(0, 1), (7, 31), (62, 63), (40, 45)]:
        a = O.pair_term(*args, i, j, omega=omega)
        b = O.pair_term(*args, j, i, omega=omega)
        assert np.array_equal(a[:3], -b[:3]) and a[3] == b[3]


def test_state_grad_h_switch_changes_only_forces():
    from paper_1905_03344_amd import inputs
    ps = inputs.square_patch(8, 1)
    s0 = O.State(ps, O.Params())
    s1 = O.State(ps, O.Params(grad_h=True))
    s0.evaluate()
    s1.evaluate()
    np.testing.assert_array_equal(s0.f["rho"], s1.f["rho"])
    assert np.all(s1.omega > 0.5) and np.all(s1.omega < 1.5)
    assert not np.array_equal(s0.f["ax"], s1.f["ax"])


def test_plain_energy_rate_is_adiabatic_with_unequal_pressures():
    """The plain (kernel-averaged) energy equation at one common, fixed h:
    there grad W_bar = grad_i W(r, h), so du_i must equal
    (P_i / rho_i^2) d rho_i / dt, the first law of an adiabatic gas, with
    d rho_i / dt a central difference of the brute-force density sum along
    the velocity field.  Each particle has its own u, so pressures differ
    pair by pair: taking P_j / rho_j^2 (or a mean) in place of P_i / rho_i^2
    fails this check."""
    pos, m = _cloud(seed=11)
    n = len(m)
    h = np.full(n, 1.25)
    rng = np.random.default_rng(17)
    vel = rng.standard_normal(pos.shape)
    u = 0.3 + 2.0 * rng.random(n)
    off, idx = _all_pairs(n)
    rho, divv = O.density(*pos.T, *vel.T, m, h, (0, 0, 0), (0, 0, 0), (0, 0, 0), off, idx)
    np.testing.assert_allclose(rho, _rho_of(pos, m, h), rtol=1e-13)
    P, c = O.eos(rho, u)
    ratio = P / rho ** 2
    assert np.max(ratio) > 3.0 * np.min(ratio)
    ax, ay, az, du, dt_i, amag = O.forces(*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0),
                                          (0, 0, 0), off, idx, alpha=0.0, beta=0.0)
    eps = 1e-6
    drho = (_rho_of(pos + eps * vel, m, h) - _rho_of(pos - eps * vel, m, h)) / (2 * eps)
    expect = ratio * drho
    np.testing.assert_allclose(du, expect, rtol=0, atol=1e-7 * np.max(np.abs(expect)))
    assert np.max(np.abs(expect)) > 1e-2


def test_plain_force_is_energy_gradient_at_fixed_h():
    """At one common, fixed h the plain momentum equation is the exact
    gradient of the thermal energy of an adiabatic gas, m_i a_i = -dE/dx_i
    with E = sum_k m_k K rho_k^(gamma-1) / (gamma-1); densities (hence
    pressures) differ across the cloud, so both pressure terms are checked
    pair by pair."""
    pos, m = _cloud(seed=4)
    n = len(m)
    h = np.full(n, 1.25)
    vel = np.zeros_like(pos)
    off, idx = _all_pairs(n)
    rho, _ = O.density(*pos.T, *vel.T, m, h, (0, 0, 0), (0, 0, 0), (0, 0, 0), off, idx)
    P = K_ADIA * rho ** GAMMA
    c = np.sqrt(GAMMA * P / rho)
    assert np.max(P) > 3.0 * np.min(P)
    ax, ay, az, *_ = O.forces(*pos.T, *vel.T, m, h, rho, P, c, (0, 0, 0), (0, 0, 0), (0, 0, 0),
                              off, idx, alpha=0.0, beta=0.0)
    a = np.stack([ax, ay, az], 1)

    def energy(p):
        r = _rho_of(p, m, h)
        return np.sum(m * K_ADIA * r ** (GAMMA - 1) / (GAMMA - 1))

    eps = 1e-6
    rng = np.random.default_rng(2)
    worst = 0.0
    for i in rng.choice(n, 16, replace=False):
        for d in range(3):
            pp, pm = pos.copy(), pos.copy()
            pp[i, d] += eps
            pm[i, d] -= eps
            g = -(energy(pp) - energy(pm)) / (2 * eps) / m[i]
            worst = max(worst, abs(a[i, d] - g))
    assert worst < 1e-6 * np.max(np.abs(a))
