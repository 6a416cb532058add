"""Seeded synthetic inputs: particle initial conditions and MLP test data.

This module holds only random-number generation and input construction; it
contains none of the SPH method's arithmetic (no kernel, neighbour test,
density, force or integrator).  Both the GPU path and the CPU oracle are fed
the arrays built here.

Generators
----------
* SplitMix64 (Steele, Lea & Flood 2014) used as a counter-based generator:
  value(seed, c) = mix64(seed + (c + 1) * 0x9E3779B97F4A7C15), and a uniform
  double in [0, 1) is (value >> 11) * 2**-53.
* Rotating square patch (the paper's test case, section "Status of the
  Mini-App", Table 3 and the rigid-rotation velocity equation): a 2D
  n_side x n_side square in x-y, copied n_side times along z, with periodic
  boundaries in z.  Cell-centred lattice in [-0.5, 0.5)^3, each coordinate
  jittered by U[-0.01 s, 0.01 s).  Velocity 5 * (-y, x, 0), u = 1, equal
  masses 1/N (density 1).
* Clumpy mixture for the learned smoothing length: 64 isotropic Gaussian
  clumps plus a 20 % uniform background in the unit cube, open boundaries.

Every array is returned as a NumPy array in "id" order (particle id i is row i).
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field

import numpy as np

GOLDEN_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# stream offsets keep independent draws of one config apart (counter space)
STREAM_STRIDE = 1 << 40


def splitmix64(seed: int, counters: np.ndarray) -> np.ndarray:
    """Counter-based SplitMix64: 64-bit output for each counter value."""
    c = np.asarray(counters, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (c + np.uint64(1)) * GOLDEN_GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, counters: np.ndarray) -> np.ndarray:
    """Uniform doubles in [0, 1): top 53 bits of SplitMix64 times 2**-53."""
    z = splitmix64(seed, counters)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def _stream(seed: int, stream: int, n: int, start: int = 0) -> np.ndarray:
    c = np.arange(start, start + n, dtype=np.uint64) + np.uint64(stream * STREAM_STRIDE)
    return uniform01(seed, c)


def gaussian(seed: int, stream: int, n: int) -> np.ndarray:
    """Standard normal draws by Box-Muller on two uniform streams."""
    u1 = _stream(seed, stream, n)
    u2 = _stream(seed, stream + 1, n)
    u1 = 1.0 - u1  # (0, 1]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * math.pi * u2)


@dataclass
class ParticleSet:
    """Initial conditions in id order, plus the box description."""
    x: np.ndarray
    y: np.ndarray
    z: np.ndarray
    vx: np.ndarray
    vy: np.ndarray
    vz: np.ndarray
    m: np.ndarray
    h: np.ndarray
    u: np.ndarray
    periodic: tuple = (0, 0, 0)
    box_lo: tuple = (0.0, 0.0, 0.0)
    box_hi: tuple = (0.0, 0.0, 0.0)
    name: str = ""
    meta: dict = field(default_factory=dict)

    @property
    def n(self) -> int:
        return int(self.x.shape[0])

    def arrays(self) -> dict:
        return {k: getattr(self, k) for k in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u")}

    def copy(self) -> "ParticleSet":
        return ParticleSet(**{k: v.copy() for k, v in self.arrays().items()},
                           periodic=self.periodic, box_lo=self.box_lo, box_hi=self.box_hi,
                           name=self.name, meta=dict(self.meta))

    def subset(self, idx: np.ndarray) -> "ParticleSet":
        return ParticleSet(**{k: v[idx].copy() for k, v in self.arrays().items()},
                           periodic=self.periodic, box_lo=self.box_lo, box_hi=self.box_hi,
                           name=self.name + "_sub", meta=dict(self.meta))


def initial_h(number_density, n_target: float = 100.0) -> np.ndarray:
    """Initial smoothing-length guess: a sphere of radius 2h holding n_target
    particles at the given number density, h0 = 0.5 (3 n_target / (4 pi n))^(1/3)."""
    nd = np.asarray(number_density, dtype=np.float64)
    return 0.5 * np.cbrt(3.0 * n_target / (4.0 * math.pi * nd))


def square_patch(n_side: int, seed: int, jitter: float = 0.01, omega: float = 5.0,
                 n_target: float = 100.0, spacing: float | None = None) -> ParticleSet:
    """Rotating square patch: n_side^3 particles in [-0.5, 0.5)^3, periodic in z.
    With `spacing` the lattice keeps that spacing (and density 1) and the box
    shrinks to n_side * spacing: a cut-out of a larger patch with the same
    per-particle work."""
    n = n_side ** 3
    s = 1.0 / n_side if spacing is None else float(spacing)
    half = 0.5 * n_side * s
    pid = np.arange(n, dtype=np.int64)
    i = pid % n_side
    j = (pid // n_side) % n_side
    k = pid // (n_side * n_side)
    cnt = 3 * pid.astype(np.uint64)
    jx = (2.0 * uniform01(seed, cnt) - 1.0) * (jitter * s)
    jy = (2.0 * uniform01(seed, cnt + np.uint64(1)) - 1.0) * (jitter * s)
    jz = (2.0 * uniform01(seed, cnt + np.uint64(2)) - 1.0) * (jitter * s)
    x = -half + (i + 0.5) * s + jx
    y = -half + (j + 0.5) * s + jy
    z = -half + (k + 0.5) * s + jz
    vx = -omega * y
    vy = omega * x
    vz = np.zeros(n)
    m = np.full(n, s ** 3) if spacing is not None else np.full(n, 1.0 / n)
    h = np.full(n, float(initial_h(1.0 / s ** 3, n_target)))
    u = np.ones(n)
    return ParticleSet(x, y, z, vx, vy, vz, m, h, u, periodic=(0, 0, 1),
                       box_lo=(-half, -half, -half), box_hi=(half, half, half),
                       name=f"square_patch_{n_side}^3", meta={"seed": seed, "s": s})


def perfect_lattice(n_side: int, h_over_s: float = 1.5, periodic_all: bool = True) -> ParticleSet:
    """Unjittered cubic lattice in [0, 1)^3 with unit total mass (density 1),
    at rest, u = 1.  Periodic in all three dimensions by default."""
    n = n_side ** 3
    s = 1.0 / n_side
    pid = np.arange(n, dtype=np.int64)
    i = pid % n_side
    j = (pid // n_side) % n_side
    k = pid // (n_side * n_side)
    x = (i + 0.5) * s
    y = (j + 0.5) * s
    z = (k + 0.5) * s
    zeros = np.zeros(n)
    per = (1, 1, 1) if periodic_all else (0, 0, 0)
    return ParticleSet(x, y, z, zeros.copy(), zeros.copy(), zeros.copy(), np.full(n, s ** 3),
                       np.full(n, h_over_s * s), np.ones(n), periodic=per,
                       box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0),
                       name=f"lattice_{n_side}^3", meta={"s": s})


def clumpy(n_clumps: int = 64, per_clump: int = 12500, n_background: int = 200000,
           seed: int = 1905033444, sigma_range=(0.02, 0.1), omega: float = 5.0,
           v_noise: float = 0.1, n_target: float = 100.0) -> ParticleSet:
    """Mixture of isotropic Gaussian clumps plus a uniform background in the
    unit cube; open boundaries.  Clump membership is in contiguous id blocks,
    the background comes last.  h starts from the mixture's analytic number
    density at each particle (the iteration then converges it)."""
    n_c = n_clumps * per_clump
    n = n_c + n_background
    # stream 0: clump parameters (4 per clump), streams 1..6: gaussians, 7: background, 8..13: v noise
    par = _stream(seed, 0, 4 * n_clumps).reshape(n_clumps, 4)
    centres = par[:, :3]
    sig = sigma_range[0] + (sigma_range[1] - sigma_range[0]) * par[:, 3]
    member = np.repeat(np.arange(n_clumps), per_clump)
    gx = gaussian(seed, 1, n_c)
    gy = gaussian(seed, 3, n_c)
    gz = gaussian(seed, 5, n_c)
    bg = _stream(seed, 7, 3 * n_background).reshape(n_background, 3)
    x = np.concatenate([centres[member, 0] + sig[member] * gx, bg[:, 0]])
    y = np.concatenate([centres[member, 1] + sig[member] * gy, bg[:, 1]])
    z = np.concatenate([centres[member, 2] + sig[member] * gz, bg[:, 2]])
    vx = -omega * (y - 0.5) + v_noise * gaussian(seed, 8, n)
    vy = omega * (x - 0.5) + v_noise * gaussian(seed, 10, n)
    vz = v_noise * gaussian(seed, 12, n)
    m = np.full(n, 1.0 / n)
    u = np.ones(n)
    # analytic number density of the mixture (in particles per unit volume)
    nd = np.zeros(n)
    inside = (x >= 0) & (x < 1) & (y >= 0) & (y < 1) & (z >= 0) & (z < 1)
    nd += n_background * inside
    for c in range(n_clumps):
        r2 = (x - centres[c, 0]) ** 2 + (y - centres[c, 1]) ** 2 + (z - centres[c, 2]) ** 2
        nd += per_clump * np.exp(-0.5 * r2 / sig[c] ** 2) / ((2 * math.pi) ** 1.5 * sig[c] ** 3)
    nd = np.maximum(nd, 1.0)
    h = initial_h(nd, n_target)
    return ParticleSet(x, y, z, vx, vy, vz, m, h, u, periodic=(0, 0, 0),
                       box_lo=(0.0, 0.0, 0.0), box_hi=(1.0, 1.0, 1.0),
                       name=f"clumpy_{n}", meta={"seed": seed, "centres": centres, "sigma": sig})


# ---------------------------------------------------------------------------
# MLP inputs (learned smoothing length): weights and synthetic feature batches
# ---------------------------------------------------------------------------

MLP_SHAPE = (6, 64, 64, 1)


def mlp_init(seed: int, shape=MLP_SHAPE) -> dict:
    """Xavier-uniform weights (row-major [out, in]) and zero biases, float32."""
    out = {}
    for layer, (fan_in, fan_out) in enumerate(zip(shape[:-1], shape[1:])):
        bound = math.sqrt(6.0 / (fan_in + fan_out))
        u = _stream(seed, 20 + layer, fan_in * fan_out)
        out[f"W{layer + 1}"] = ((2.0 * u - 1.0) * bound).astype(np.float32).reshape(fan_out, fan_in)
        out[f"b{layer + 1}"] = np.zeros(fan_out, dtype=np.float32)
    return out


def mlp_batch(seed: int, n: int, n_in: int = 6, scale: float = 1.5) -> tuple:
    """Synthetic standardised features in [-scale, scale) and targets in [-0.4, 0.4)."""
    f = ((2.0 * _stream(seed, 40, n * n_in) - 1.0) * scale).reshape(n, n_in)
    y = (2.0 * _stream(seed, 41, n) - 1.0) * 0.4
    return f, y


def shuffle_order(seed: int, n: int) -> np.ndarray:
    """A seeded permutation of 0..n-1 (int32): the order of training rows."""
    return np.argsort(_stream(seed, 60, n), kind="stable").astype(np.int32)


CONFIG_SEEDS = {1: 1905033441, 2: 1905033442, 3: 1905033443, 4: 1905033444, 5: 1905033445}


def config_ic(cfg: int, seed_offset: int = 0) -> ParticleSet:
    """Initial conditions of the five workloads (square patch 20^3, 100^3,
    200^3, clumpy 1M, square patch 400^3); seed_offset draws another sample
    of the same distribution (100: the learned form's evaluation seed)."""
    if cfg not in CONFIG_SEEDS:
        raise ValueError(f"unknown config {cfg}")
    seed = CONFIG_SEEDS[cfg] + seed_offset
    if cfg == 1:
        return square_patch(20, seed)
    if cfg == 2:
        return square_patch(100, seed)
    if cfg == 3:
        return square_patch(200, seed)
    if cfg == 4:
        return clumpy(seed=seed)
    return square_patch(400, seed)
