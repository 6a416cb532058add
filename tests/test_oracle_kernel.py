"""Pins for the oracle's smoothing kernels (kernel section of the paper: support
0 <= v <= 2; Wendland normalisation sigma_W = 21/(16 pi); the sinc family,
whose exponent and normalisation the paper does not print: exponent 5, B_5
from normalisation).

None of these re-types the oracle's formula: normalisation is checked by
numerical quadrature, smoothness by one-sided limits, the derivative by
finite differences of W, and scaling by the dimensional law W(lr, lh) =
W(r, h)/l^3."""
import math

import numpy as np
import pytest
from scipy import integrate

import oracle as O


@pytest.mark.parametrize("h", [1.0, 0.37, 2.5e-3])
def test_m4_normalisation(h):
    f = lambda r: 4.0 * math.pi * r * r * O.kernel_w(r, h)
    val, err = integrate.quad(f, 0.0, 2.0 * h, points=[h], epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12


def test_wendland_normalisation_matches_paper_constant():
    # the paper prints sigma_W = 21/(16 pi); with the 3D 1/h^3 factor the
    # volume integral of the printed kernel must be one
    h = 0.8
    f = lambda r: 4.0 * math.pi * r * r * O.kernel_wendland(r, h)
    val, _ = integrate.quad(f, 0.0, 2.0 * h, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12


def test_m4_compact_support_and_centre():
    h = 0.3
    assert O.kernel_w(2.0 * h, h) == 0.0
    assert O.kernel_w(2.5 * h, h) == 0.0
    assert O.kernel_dwdr(2.0 * h, h) == 0.0
    assert O.kernel_dwdr(0.0, h) == 0.0
    assert O.kernel_w(0.0, h) == pytest.approx(1.0 / (math.pi * h ** 3), rel=1e-15)
    # W is positive and decreasing inside the support
    r = np.linspace(0, 2 * h, 401)[:-1]
    w = np.array([O.kernel_w(v, h) for v in r])
    assert np.all(w > 0) and np.all(np.diff(w) < 0)


@pytest.mark.parametrize("q", [1.0, 2.0])
def test_m4_c1_continuity(q):
    h = 1.0
    eps = 1e-9
    wl, wr = O.kernel_w(q - eps, h), O.kernel_w(q + eps if q < 2 else q, h)
    dl, dr = O.kernel_dwdr(q - eps, h), O.kernel_dwdr(q + eps if q < 2 else q, h)
    assert abs(wl - wr) < 1e-8
    assert abs(dl - dr) < 1e-8


def test_m4_derivative_finite_difference():
    h = 0.7
    for r in np.linspace(0.01, 1.39, 57):
        e = 1e-6
        fd = (O.kernel_w(r + e, h) - O.kernel_w(r - e, h)) / (2 * e)
        assert abs(fd - O.kernel_dwdr(r, h)) < 1e-7 * (1 + abs(fd))


def test_m4_dimensional_scaling():
    for lam in (0.5, 3.0):
        for r in (0.1, 0.9, 1.5):
            assert O.kernel_w(lam * r, lam * 1.0) == pytest.approx(O.kernel_w(r, 1.0) / lam ** 3,
                                                                     rel=1e-14)
            assert O.kernel_dwdr(lam * r, lam) == pytest.approx(O.kernel_dwdr(r, 1.0) / lam ** 4,
                                                                  rel=1e-14)


def test_hk_table():
    T = O.hk_table(100)
    assert T[0] == 2.0
    assert T[100] == 1.0
    # (100/k)^(1/3) for a perfect cube ratio
    assert T[800] == pytest.approx(0.5 * (1 + 0.5), rel=1e-15)
    assert np.all(T >= 0.5) and np.all(T <= 2.0)
    assert np.all(np.diff(T[1:]) <= 0)


# --- Wendland C2 and sinc (n = 5): the kernel section's own kernels ---------

KERNELS = {"wendland": (O.kernel_wendland, O.kernel_wendland_dwdr),
           "sinc5": (O.kernel_sinc, O.kernel_sinc_dwdr)}


@pytest.mark.parametrize("name", sorted(KERNELS))
@pytest.mark.parametrize("h", [1.0, 0.37])
def test_normalisation(name, h):
    w, _ = KERNELS[name]
    f = lambda r: 4.0 * math.pi * r * r * w(r, h)
    val, _ = integrate.quad(f, 0.0, 2.0 * h, epsabs=0, epsrel=1e-13, limit=200)
    assert abs(val - 1.0) < 1e-12


@pytest.mark.parametrize("name", sorted(KERNELS))
def test_derivative_finite_difference(name):
    w, dw = KERNELS[name]
    h = 0.7
    for r in np.linspace(0.003, 1.397, 71):
        e = 1e-6
        fd = (w(r + e, h) - w(r - e, h)) / (2 * e)
        assert abs(fd - dw(r, h)) < 1e-7 * (1 + abs(fd)), (name, r)


@pytest.mark.parametrize("name", sorted(KERNELS))
def test_support_end_and_centre(name):
    w, dw = KERNELS[name]
    h = 0.3
    assert w(2.0 * h, h) == 0.0 and dw(2.0 * h, h) == 0.0
    assert dw(0.0, h) == 0.0
    # both vanish smoothly at the support end (C1 or better): values just
    # inside are tiny compared with the centre
    assert w(2.0 * h * (1 - 1e-4), h) < 1e-10 * w(0.0, h)
    assert abs(dw(2.0 * h * (1 - 1e-4), h)) < 1e-6 * abs(dw(h, h))
    # positive and decreasing inside the support
    r = np.linspace(0, 2 * h, 401)[:-1]
    vals = np.array([w(v, h) for v in r])
    assert np.all(vals > 0) and np.all(np.diff(vals) < 0)


@pytest.mark.parametrize("name", sorted(KERNELS))
def test_dimensional_scaling(name):
    w, dw = KERNELS[name]
    for lam in (0.5, 3.0):
        for r in (0.1, 0.9, 1.5):
            assert w(lam * r, lam) == pytest.approx(w(r, 1.0) / lam ** 3, rel=1e-14)
            assert dw(lam * r, lam) == pytest.approx(dw(r, 1.0) / lam ** 4, rel=1e-14)


def test_wendland_centre_is_paper_constant():
    # W(0, h) = sigma_W / h^3 with the printed sigma_W = 21 / (16 pi)
    assert O.kernel_wendland(0.0, 2.0) == pytest.approx(21.0 / (16.0 * math.pi) / 8.0, rel=1e-15)


def test_sinc_shape_and_series_switch():
    # the shape against numpy's own sinc, np.sinc(t) = sin(pi t)/(pi t):
    # W(r, 1) / W(0, 1) = np.sinc(v/2)^5, across the series/direct switch of
    # the oracle's evaluation (x = pi v / 2 = 1/2)
    b = O.kernel_sinc(0.0, 1.0)
    assert b == pytest.approx(O.sinc_norm(), rel=1e-15)
    for v in np.concatenate([np.linspace(0.0, 1.99, 200), [1 / math.pi - 1e-12, 1 / math.pi]]):
        assert O.kernel_sinc(v, 1.0) == pytest.approx(b * np.sinc(v / 2.0) ** 5, rel=1e-13,
                                                     abs=1e-300)
    # the derivative is continuous across the switch
    v0 = 1.0 / math.pi
    assert O.kernel_sinc_dwdr(v0 * (1 - 1e-12), 1.0) == pytest.approx(
        O.kernel_sinc_dwdr(v0 * (1 + 1e-12), 1.0), rel=1e-9)
