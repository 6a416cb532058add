"""CPU FP64 oracle for the SPH step -- TEST INFRASTRUCTURE ONLY.

Only the test suite, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  It never imports the GPU package and
the GPU package never imports it; both take their inputs from the seeded
generators in ``paper_1905_03344_amd.inputs``.

The arithmetic lives in ``sph_oracle.c`` (plain C, one IEEE operation at a
time, no FMA contraction); this module is argument marshalling plus the
composition of the stages into one kick-drift-kick step, in the order:
kick + drift, bounding box, cell keys, stable sort, permutation, prediction,
smoothing-length iteration, interaction lists, density + divergence, EOS,
momentum + energy + viscosity + Courant step, second kick.

Parity status per function (all pinned in tests/test_oracle_*.py):
kernel -- quadrature, continuity, finite differences;
keys/sort -- an independent Python re-derivation and numpy's stable argsort;
counts/lists -- brute force O(N^2) and set symmetry;
h iteration -- band membership and the lattice non-convergence case;
density/divergence -- lattice closed forms, two-particle closed form, rigid
rotation; EOS -- closed form; forces -- antisymmetry and conservation laws,
Galilean invariance, uniform-lattice equilibrium; integrator -- exactness
for constant acceleration and second-order convergence; grad-h terms --
finite-difference derivatives of the thermal energy with h solved
self-consistently; IAD matrices -- inverse of a brute-force moment sum and
exact gradients of linear fields, IAD forces -- closed forms on a lattice
under linear pressure and velocity fields; MLP -- finite differences.  None of these quantities is published in the paper, so no
value is pinned to a printed number.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None

_d = ctypes.POINTER(ctypes.c_double)
_i32 = ctypes.POINTER(ctypes.c_int32)
_i64 = ctypes.POINTER(ctypes.c_int64)
_u32 = ctypes.POINTER(ctypes.c_uint32)
_u8 = ctypes.POINTER(ctypes.c_uint8)
_int3 = ctypes.c_int * 3
_dbl3 = ctypes.c_double * 3


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB_PATH):
            from . import build as _b
            _b.build()
        L = ctypes.CDLL(_LIB_PATH)
        L.or_kernel_w.restype = ctypes.c_double
        L.or_kernel_w.argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_kernel_dwdr.restype = ctypes.c_double
        L.or_kernel_dwdr.argtypes = [ctypes.c_double, ctypes.c_double]
        for nm in ("or_kernel_wendland", "or_kernel_wendland_dwdr", "or_kernel_sinc",
                   "or_kernel_sinc_dwdr"):
            getattr(L, nm).restype = ctypes.c_double
            getattr(L, nm).argtypes = [ctypes.c_double, ctypes.c_double]
        L.or_sinc_norm.restype = ctypes.c_double
        L.or_sinc_norm.argtypes = []
        L.or_kernel_dwdh.restype = ctypes.c_double
        L.or_kernel_dwdh.argtypes = [ctypes.c_int, ctypes.c_double, ctypes.c_double]
        L.or_hsolve.restype = ctypes.c_int64
        L.or_iad.restype = ctypes.c_int64
        L.or_lists.restype = ctypes.c_int64
        L.or_mlp_loss_grad.restype = ctypes.c_double
        L.or_num_threads.restype = ctypes.c_int
        _lib = L
    return _lib


def _p(a, t=_d):
    return a.ctypes.data_as(t)


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


# ---------------------------------------------------------------------------
# elementary functions
# ---------------------------------------------------------------------------

def kernel_w(r, h):
    return lib().or_kernel_w(float(r), float(h))


def kernel_dwdr(r, h):
    return lib().or_kernel_dwdr(float(r), float(h))


def kernel_wendland(r, h):
    return lib().or_kernel_wendland(float(r), float(h))


def kernel_wendland_dwdr(r, h):
    return lib().or_kernel_wendland_dwdr(float(r), float(h))


def kernel_sinc(r, h):
    """sinc kernel, exponent 5 (kernel section; B_5 by normalisation)"""
    return lib().or_kernel_sinc(float(r), float(h))


def kernel_sinc_dwdr(r, h):
    return lib().or_kernel_sinc_dwdr(float(r), float(h))


def sinc_norm():
    return lib().or_sinc_norm()


def kernel_dwdh(r, h, kernel=0):
    """dW/dh at fixed r (grad-h factor)"""
    return lib().or_kernel_dwdh(int(kernel), float(r), float(h))


# kernel ids of the density and force sums (same numbering as the library's
# sph_params.kernel)
KERNEL_M4, KERNEL_WENDLAND, KERNEL_SINC5 = 0, 1, 2
# integrators: kick-drift-kick leapfrog; KDK positions and velocities with
# the energy by second-order Adams-Bashforth
INTEGRATOR_KDK, INTEGRATOR_AB2 = 0, 1
# gradient estimators of the momentum and energy sums: kernel derivatives, or
# the integral approach to derivatives (IAD)
GRADIENTS_KERNEL, GRADIENTS_IAD = 0, 1
# volume elements of the density sum (Table 1): standard (X = m) or generalized,
# X_i = (m_i / rho_i)^p from the previous evaluation's density
VOLUMES_STANDARD, VOLUMES_GENERALIZED = 0, 1


def ab2_energy(u, du, du_prev, dt, dt_prev, hist):
    """u after one Adams-Bashforth step (Euler without history)."""
    u = _f64(u).copy()
    du = _f64(du)
    dup = _f64(du_prev if du_prev is not None else du)
    lib().or_ab2_energy(ctypes.c_int64(len(u)), ctypes.c_double(dt), ctypes.c_double(dt_prev),
                        ctypes.c_int(int(hist)), _p(u), _p(du), _p(dup))
    return u


def hk_table(n_target=100):
    T = np.zeros(1024)
    lib().or_hk_table(ctypes.c_int(n_target), _p(T))
    return T


def num_threads():
    return lib().or_num_threads()


def set_num_threads(n: int):
    """Thread count of the oracle's later parallel loops (for timing)."""
    lib().or_set_num_threads(ctypes.c_int(int(n)))


# ---------------------------------------------------------------------------
# geometry: bounding box, keys, sort, cell tables
# ---------------------------------------------------------------------------

def bbox(x, y, z, periodic, box_lo, box_hi):
    lo = np.zeros(3)
    hi = np.zeros(3)
    x, y, z = _f64(x), _f64(y), _f64(z)
    lib().or_bbox(ctypes.c_int64(len(x)), _p(x), _p(y), _p(z), _int3(*periodic),
                  _dbl3(*box_lo), _dbl3(*box_hi), _p(lo), _p(hi))
    return lo, hi


def cell_keys(x, y, z, lo, hi):
    x, y, z = _f64(x), _f64(y), _f64(z)
    key = np.zeros(len(x), dtype=np.uint32)
    lo = _f64(lo)
    hi = _f64(hi)
    lib().or_cell_keys(ctypes.c_int64(len(x)), _p(x), _p(y), _p(z), _p(lo), _p(hi), _p(key, _u32))
    return key


def sort_perm(key):
    key = np.ascontiguousarray(key, dtype=np.uint32)
    perm = np.zeros(len(key), dtype=np.int32)
    lib().or_sort_perm(ctypes.c_int64(len(key)), _p(key, _u32), _p(perm, _i32))
    return perm


def cell_start(sorted_key, level):
    sorted_key = np.ascontiguousarray(sorted_key, dtype=np.uint32)
    start = np.zeros((1 << (3 * level)) + 1, dtype=np.int32)
    lib().or_cell_start(ctypes.c_int64(len(sorted_key)), _p(sorted_key, _u32), ctypes.c_int(level),
                        _p(start, _i32))
    return start


# ---------------------------------------------------------------------------
# neighbours and smoothing length
# ---------------------------------------------------------------------------

def count(x, y, z, h, periodic, box_lo, box_hi, method=1):
    x, y, z, h = _f64(x), _f64(y), _f64(z), _f64(h)
    out = np.zeros(len(x), dtype=np.int32)
    lib().or_count(ctypes.c_int64(len(x)), _p(x), _p(y), _p(z), _p(h), _int3(*periodic),
                   _dbl3(*box_lo), _dbl3(*box_hi), ctypes.c_int(method), _p(out, _i32))
    return out


def hsolve(x, y, z, h_in, periodic, box_lo, box_hi, n_target=100, n_tol=5, max_iter=32,
           method=1):
    x, y, z, h_in = _f64(x), _f64(y), _f64(z), _f64(h_in)
    n = len(x)
    h = np.zeros(n)
    nc = np.zeros(n, dtype=np.int32)
    flag = np.zeros(n, dtype=np.uint8)
    iters = np.zeros(n, dtype=np.int32)
    nonconv = lib().or_hsolve(ctypes.c_int64(n), _p(x), _p(y), _p(z), _p(h_in), _int3(*periodic),
                              _dbl3(*box_lo), _dbl3(*box_hi), ctypes.c_int(n_target),
                              ctypes.c_int(n_tol), ctypes.c_int(max_iter), ctypes.c_int(method),
                              _p(h), _p(nc, _i32), _p(flag, _u8), _p(iters, _i32))
    return h, nc, flag, iters, int(nonconv)


def lists(x, y, z, h, periodic, box_lo, box_hi, method=1, symmetric=True):
    """Interaction sets S (symmetric) or gather sets L, CSR with ascending rows."""
    x, y, z, h = _f64(x), _f64(y), _f64(z), _f64(h)
    n = len(x)
    off = np.zeros(n + 1, dtype=np.int64)
    idx_ptr = ctypes.POINTER(ctypes.c_int32)()
    total = lib().or_lists(ctypes.c_int64(n), _p(x), _p(y), _p(z), _p(h), _int3(*periodic),
                           _dbl3(*box_lo), _dbl3(*box_hi), ctypes.c_int(method),
                           ctypes.c_int(int(symmetric)), _p(off, _i64), ctypes.byref(idx_ptr))
    idx = np.ctypeslib.as_array(idx_ptr, shape=(max(total, 1),))[:total].copy()
    lib().or_free(idx_ptr)
    return off, idx


# ---------------------------------------------------------------------------
# fields
# ---------------------------------------------------------------------------

def density(x, y, z, vx, vy, vz, m, h, periodic, box_lo, box_hi, off, idx, with_mag=False,
            kernel=0, with_omega=False, X=None, with_ysum=False):
    """rho, divv (and, with_mag, (1/rho) sum |m_j (v_j - v_i).grad W|, the scale
    of the divergence sum used for conditioning-aware comparisons; with_omega
    also the grad-h factors Omega; with_ysum the weighted sum Y, appended in
    that order).  X: the weights of generalized volume elements (None: the
    standard density, X = m)."""
    arr = [_f64(a) for a in (x, y, z, vx, vy, vz, m, h)]
    n = len(arr[0])
    rho = np.zeros(n)
    divv = np.zeros(n)
    mag = np.zeros(n)
    om = np.zeros(n)
    ys = np.zeros(n)
    off = np.ascontiguousarray(off, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    Xa = _f64(X) if X is not None else None
    lib().or_density(ctypes.c_int64(n), *[_p(a) for a in arr], _int3(*periodic), _dbl3(*box_lo),
                     _dbl3(*box_hi), _p(off, _i64), _p(idx, _i32), _p(rho), _p(divv), _p(mag),
                     ctypes.c_int(kernel), _p(om), _p(Xa) if Xa is not None else None, _p(ys))
    out = (rho, divv, mag) if with_mag else (rho, divv)
    if with_omega:
        out = out + (om,)
    return out + (ys,) if with_ysum else out


def eos(rho, u, gamma=5.0 / 3.0):
    rho, u = _f64(rho), _f64(u)
    p = np.zeros(len(rho))
    c = np.zeros(len(rho))
    lib().or_eos(ctypes.c_int64(len(rho)), _p(rho), _p(u), ctypes.c_double(gamma), _p(p), _p(c))
    return p, c


def forces(x, y, z, vx, vy, vz, m, h, rho, p, c, periodic, box_lo, box_hi, off, idx,
           alpha=1.0, beta=2.0, eta2=0.01, cfl=0.3, with_mag=False, kernel=0, omega=None,
           iad=None, gve=None):
    """a, du, per-particle dt, sum_j m_j |f_ij| (and with_mag sum_j m_j |de_ij|).
    gve: (X/m, P/Y^2) per particle for generalized volume elements."""
    arr = [_f64(a) for a in (x, y, z, vx, vy, vz, m, h, rho, p, c)]
    n = len(arr[0])
    out = [np.zeros(n) for _ in range(7)]
    off = np.ascontiguousarray(off, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    lib().or_forces(ctypes.c_int64(n), *[_p(a) for a in arr], _int3(*periodic), _dbl3(*box_lo),
                    _dbl3(*box_hi), _p(off, _i64), _p(idx, _i32), ctypes.c_double(alpha),
                    ctypes.c_double(beta), ctypes.c_double(eta2), ctypes.c_double(cfl),
                    *[_p(a) for a in out], ctypes.c_int(kernel),
                    _p(_f64(omega)) if omega is not None else None,
                    _p(_f64(iad)) if iad is not None else None,
                    *_gve_ptrs(gve))
    ax, ay, az, du, dt_i, amag, dumag = out
    if with_mag:
        return ax, ay, az, du, dt_i, amag, dumag
    return ax, ay, az, du, dt_i, amag


_gve_keep = []


def _gve_ptrs(gve):
    if gve is None:
        return None, None
    r, g = _f64(gve[0]), _f64(gve[1])
    _gve_keep[:] = [r, g]   # alive for the duration of the call
    return _p(r), _p(g)


def pair_term(x, y, z, vx, vy, vz, m, h, rho, p, c, periodic, box_lo, box_hi, i, j,
              alpha=1.0, beta=2.0, eta2=0.01, kernel=0, omega=None, iad=None, gve=None):
    arr = [_f64(a) for a in (x, y, z, vx, vy, vz, m, h, rho, p, c)]
    out = np.zeros(4)
    lib().or_pair_term(ctypes.c_int64(len(arr[0])), *[_p(a) for a in arr], _int3(*periodic),
                       _dbl3(*box_lo), _dbl3(*box_hi), ctypes.c_int64(i), ctypes.c_int64(j),
                       ctypes.c_double(alpha), ctypes.c_double(beta), ctypes.c_double(eta2),
                       _p(out), ctypes.c_int(kernel),
                       _p(_f64(omega)) if omega is not None else None,
                       _p(_f64(iad)) if iad is not None else None,
                       *_gve_ptrs(gve))
    return out


def iad_matrices(x, y, z, m, rho, h, periodic, box_lo, box_hi, off, idx, kernel=0):
    """IAD inverse moment matrices c_i, (n, 6) as (xx, xy, xz, yy, yz, zz),
    and the count of singular ones (left NaN)."""
    arr = [_f64(a) for a in (x, y, z, m, rho, h)]
    n = len(arr[0])
    out = np.zeros((n, 6))
    off = np.ascontiguousarray(off, dtype=np.int64)
    idx = np.ascontiguousarray(idx, dtype=np.int32)
    bad = lib().or_iad(ctypes.c_int64(n), *[_p(a) for a in arr], _int3(*periodic), _dbl3(*box_lo),
                       _dbl3(*box_hi), _p(off, _i64), _p(idx, _i32), ctypes.c_int(kernel),
                       _p(out))
    return out, int(bad)


def conservation(x, y, z, vx, vy, vz, m, u):
    arr = [_f64(a) for a in (x, y, z, vx, vy, vz, m, u)]
    out = np.zeros(7)
    lib().or_conservation(ctypes.c_int64(len(arr[0])), *[_p(a) for a in arr], _p(out))
    return out


# ---------------------------------------------------------------------------
# the full step
# ---------------------------------------------------------------------------

CARRIED = ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u", "ax", "ay", "az", "du", "rho",
           "divv", "nc", "id")


@dataclass
class Params:
    n_target: int = 100
    n_tol: int = 5
    max_iter: int = 32
    gamma: float = 5.0 / 3.0
    alpha: float = 1.0
    beta: float = 2.0
    eta2: float = 0.01
    cfl: float = 0.3
    kernel: int = 0   # KERNEL_M4, KERNEL_WENDLAND or KERNEL_SINC5
    integrator: int = 0   # INTEGRATOR_KDK or INTEGRATOR_AB2
    grad_h: bool = False  # grad-h correction terms in the momentum and energy equations
    gradients: int = 0    # GRADIENTS_KERNEL or GRADIENTS_IAD
    volumes: int = 0      # VOLUMES_STANDARD or VOLUMES_GENERALIZED
    gve_exponent: float = 0.7   # p of the generalized weights X = (m / rho)^p


class State:
    """Particle state in storage order (after the latest sort)."""

    def __init__(self, ic, params: Params | None = None):
        self.p = params or Params()
        self.periodic = tuple(int(v) for v in ic.periodic)
        self.box_lo = tuple(float(v) for v in ic.box_lo)
        self.box_hi = tuple(float(v) for v in ic.box_hi)
        n = ic.n
        self.f = {k: np.array(v, dtype=np.float64, copy=True) for k, v in ic.arrays().items()}
        for k in ("ax", "ay", "az", "du", "rho", "divv"):
            self.f[k] = np.zeros(n)
        self.f["nc"] = np.zeros(n, dtype=np.int32)
        self.f["id"] = np.arange(n, dtype=np.int32)
        self.pv = None  # predicted velocities / energy used by the last evaluation
        self.dt_next = None
        self.off = None
        self.idx = None
        self.keys = None
        self.perm = None
        self.flags = None
        self.nonconv = 0
        self.keep_gather = False
        # smoothing lengths to evaluate at instead of solving for them (in
        # the order after the next sort); used to check a form that chose
        # its own in-band h against these same stages at that h
        self.h_given = None
        self.dt_prev = None     # the previous step's dt (Adams-Bashforth energy)

    @property
    def n(self):
        return len(self.f["x"])

    def geom(self):
        return self.periodic, self.box_lo, self.box_hi

    # --- stages -----------------------------------------------------------
    def build_cells(self):
        f = self.f
        lo, hi = bbox(f["x"], f["y"], f["z"], *self.geom())
        key = cell_keys(f["x"], f["y"], f["z"], lo, hi)
        perm = sort_perm(key)
        for k in CARRIED + (("du_prev",) if "du_prev" in f else ()):
            f[k] = f[k][perm].copy()
        self.keys = key[perm]
        self.perm = perm
        self.lo, self.hi = lo, hi
        return perm

    def find_neighbors(self, method=1):
        f = self.f
        if self.h_given is not None:
            h = _f64(self.h_given).copy()
            nc = count(f["x"], f["y"], f["z"], h, *self.geom(), method)
            flag = np.zeros(self.n, dtype=np.uint8)
            iters, nonconv = np.zeros(self.n, dtype=np.int32), 0
            self.h_given = None
        else:
            h, nc, flag, iters, nonconv = hsolve(f["x"], f["y"], f["z"], f["h"], *self.geom(),
                                                 self.p.n_target, self.p.n_tol, self.p.max_iter,
                                                 method)
        f["h"], f["nc"] = h, nc
        self.flags, self.iters, self.nonconv = flag, iters, nonconv
        self.off, self.idx = lists(f["x"], f["y"], f["z"], h, *self.geom(), method)
        if self.keep_gather:
            self.loff, self.lidx = lists(f["x"], f["y"], f["z"], h, *self.geom(), method,
                                         symmetric=False)

    def evaluate(self, method=1):
        """Cells, neighbours, density, EOS and forces at the stored state
        (the force evaluation at t = 0).  Returns the Courant dt."""
        f = self.f
        f.pop("du_prev", None)   # an evaluation starts the integrator afresh
        self.dt_prev = None
        self.build_cells()
        self._evaluate_sorted((f["vx"], f["vy"], f["vz"]), f["u"], method, fresh=True)
        return self.dt_next

    def step(self, dt=None, method=1):
        """One kick-drift-kick step; dt None uses the Courant value from the
        previous evaluation."""
        if dt is None or dt <= 0:
            dt = self.dt_next
        f = self.f
        ab2 = self.p.integrator == INTEGRATOR_AB2
        if ab2:
            hist = "du_prev" in f
            u_new = ab2_energy(f["u"], f["du"], f.get("du_prev"), dt,
                               self.dt_prev if hist else 0.0, hist)
            du_n = f["du"].copy()
        vx, vy, vz, u = f["vx"].copy(), f["vy"].copy(), f["vz"].copy(), f["u"].copy()
        x, y, z = f["x"].copy(), f["y"].copy(), f["z"].copy()
        n = self.n
        lib().or_kick_drift(ctypes.c_int64(n), ctypes.c_double(dt), _p(x), _p(y), _p(z), _p(vx),
                            _p(vy), _p(vz), _p(u), _p(f["ax"]), _p(f["ay"]), _p(f["az"]),
                            _p(f["du"]), _int3(*self.periodic), _dbl3(*self.box_lo),
                            _dbl3(*self.box_hi))
        if ab2:
            u = u_new   # the energy is final at the step's start: no half kicks
            f["du_prev"] = du_n
        f["x"], f["y"], f["z"], f["vx"], f["vy"], f["vz"], f["u"] = x, y, z, vx, vy, vz, u
        # permutation happens inside evaluate; predicted values use the
        # permuted half-step state and old accelerations
        self.build_cells()
        pvx, pvy, pvz, pu = (np.zeros(n) for _ in range(4))
        lib().or_predict(ctypes.c_int64(n), ctypes.c_double(dt), _p(f["vx"]), _p(f["vy"]),
                         _p(f["vz"]), _p(f["u"]), _p(f["ax"]), _p(f["ay"]), _p(f["az"]),
                         _p(f["du"]), _p(pvx), _p(pvy), _p(pvz), _p(pu))
        if ab2:
            pu = f["u"].copy()
        self._evaluate_sorted((pvx, pvy, pvz), pu, method)
        u_keep = f["u"].copy()
        lib().or_kick(ctypes.c_int64(n), ctypes.c_double(dt), _p(f["vx"]), _p(f["vy"]),
                      _p(f["vz"]), _p(f["u"]), _p(f["ax"]), _p(f["ay"]), _p(f["az"]), _p(f["du"]))
        if ab2:
            f["u"] = u_keep
            self.dt_prev = dt
        return dt

    def gve_weights(self, rho_prev):
        """X_i = (m_i / rho_i)^p of generalized volume elements."""
        return np.power(self.f["m"] / rho_prev, self.p.gve_exponent)

    def _evaluate_sorted(self, vel, u, method, fresh=False):
        f = self.f
        self.pv = (vel, u)
        self.find_neighbors(method)
        X = None
        if self.p.volumes == VOLUMES_GENERALIZED:
            # the weights come from the previous evaluation's density; an
            # evaluation that starts a run takes the standard density first
            rho_prev = f["rho"]
            if fresh:
                rho_prev, _ = density(f["x"], f["y"], f["z"], *vel, f["m"], f["h"], *self.geom(),
                                      self.off, self.idx, kernel=self.p.kernel)
            X = self.gve_weights(rho_prev)
        rho, divv, dvmag, omega, ysum = density(f["x"], f["y"], f["z"], *vel, f["m"], f["h"],
                                                *self.geom(), self.off, self.idx, with_mag=True,
                                                kernel=self.p.kernel, with_omega=True, X=X,
                                                with_ysum=True)
        self.omega = omega
        self.X, self.ysum = X, ysum
        f["rho"], f["divv"] = rho, divv
        self.divv_mag = dvmag
        P, c = eos(rho, u, self.p.gamma)
        self.P, self.c = P, c
        gve = (X / f["m"], P / (ysum * ysum)) if X is not None else None
        self.iad = None
        if self.p.gradients == GRADIENTS_IAD:
            self.iad, bad = iad_matrices(f["x"], f["y"], f["z"], f["m"], rho, f["h"], *self.geom(),
                                         self.off, self.idx, kernel=self.p.kernel)
            if bad:
                raise FloatingPointError(f"{bad} singular IAD matrices")
        ax, ay, az, du, dt_i, amag, dumag = forces(f["x"], f["y"], f["z"], *vel, f["m"], f["h"],
                                                   rho, P, c, *self.geom(), self.off, self.idx,
                                                   self.p.alpha, self.p.beta, self.p.eta2,
                                                   self.p.cfl, with_mag=True, kernel=self.p.kernel,
                                                   omega=omega if self.p.grad_h else None,
                                                   iad=self.iad, gve=gve)
        f["ax"], f["ay"], f["az"], f["du"] = ax, ay, az, du
        self.amag, self.dumag, self.dt_i = amag, dumag, dt_i
        self.dt_next = float(dt_i.min()) if len(dt_i) else np.inf

    def conservation(self):
        f = self.f
        return conservation(f["x"], f["y"], f["z"], f["vx"], f["vy"], f["vz"], f["m"], f["u"])


# ---------------------------------------------------------------------------
# MLP
# ---------------------------------------------------------------------------

def bf16_round(a):
    a = _f64(a)
    out = np.zeros_like(a)
    lib().or_bf16_round(ctypes.c_int64(a.size), _p(a), _p(out))
    return out


def _wp(w):
    return {k: _f64(v).ravel() for k, v in w.items()}


def mlp_forward(x, w, use_bf16=True):
    """x [B, 6]; w dict W1[64,6], b1[64], W2[64,64], b2[64], W3[1,64], b3[1].
    Returns (z1, a1, z2, a2, y) in FP64; use_bf16 rounds every layer's
    operands to bfloat16 (round-to-nearest-even) as the production form does."""
    x = _f64(x).reshape(-1, 6)
    B = x.shape[0]
    W = _wp(w)
    z1, a1, z2, a2 = (np.zeros((B, 64)) for _ in range(4))
    y = np.zeros(B)
    lib().or_mlp_forward(ctypes.c_int64(B), _p(x), _p(W["W1"]), _p(W["b1"]), _p(W["W2"]),
                         _p(W["b2"]), _p(W["W3"]), _p(W["b3"]), ctypes.c_int(int(use_bf16)), _p(z1),
                         _p(a1), _p(z2), _p(a2), _p(y))
    return z1, a1, z2, a2, y


def mlp_loss_grad(x, t, w, use_bf16=True):
    x = _f64(x).reshape(-1, 6)
    t = _f64(t)
    W = _wp(w)
    g = {k: np.zeros_like(v) for k, v in W.items()}
    loss = lib().or_mlp_loss_grad(ctypes.c_int64(x.shape[0]), _p(x), _p(t), _p(W["W1"]),
                                  _p(W["b1"]), _p(W["W2"]), _p(W["b2"]), _p(W["W3"]), _p(W["b3"]),
                                  ctypes.c_int(int(use_bf16)), _p(g["W1"]), _p(g["b1"]), _p(g["W2"]), _p(g["b2"]), _p(g["W3"]),
                                  _p(g["b3"]))
    shapes = {k: np.asarray(v).shape for k, v in w.items()}
    return loss, {k: g[k].reshape(shapes[k]) for k in g}


def adam(p, m, v, g, lr=1e-3, beta1=0.9, beta2=0.999, eps=1e-8, t=1):
    p, m, v, g = (_f64(a).copy() for a in (p, m, v, g))
    shape = p.shape
    p, m, v, g = (a.ravel() for a in (p, m, v, g))
    lib().or_adam(ctypes.c_int64(p.size), _p(p), _p(m), _p(v), _p(g), ctypes.c_double(lr),
                  ctypes.c_double(beta1), ctypes.c_double(beta2), ctypes.c_double(eps),
                  ctypes.c_int(t))
    return p.reshape(shape), m.reshape(shape), v.reshape(shape)
