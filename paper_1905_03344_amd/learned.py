"""Training driver of the learned smoothing length.

The h update of the per-timestep loop (section "Co-Design of the Mini-App")
iterates h_i until the gather set of particle i holds close to the target
neighbour count.  The learned form predicts the converged h from features of
the previous step; this module harvests training rows from plain steps, fits
the feature standardisation and runs the epoch loop, all through the C ABI
(feature build, MLP forward/backward and Adam run in the library's kernels;
this file only sequences calls and owns the device buffers).

    sim = Simulation(ic_a)                  # plain mode, training trajectory
    sim.evaluate()
    feat, target = harvest(sim, steps=20)
    w, norm, losses = train(sim, feat, target, seed=...)
    sim_b = Simulation(ic_b, h_mode=ffi.SPH_H_LEARNED)
    sim_b.set_mlp(w, norm)
"""
from __future__ import annotations

import numpy as np
import torch

from . import ffi, inputs


def pack_params(w: dict) -> np.ndarray:
    """Flat FP32 parameter vector in the library's order from a dict."""
    flat = np.zeros(ffi.SPH_MLP_NPARAM, dtype=np.float32)
    for name, (off, shape) in ffi.MLP_LAYOUT.items():
        a = np.asarray(w[name], dtype=np.float32).reshape(-1)
        size = int(np.prod(shape))
        if a.size != size:
            raise ValueError(f"{name}: expected {size} values, got {a.size}")
        flat[off:off + size] = a
    return flat


def unpack_params(flat) -> dict:
    flat = np.asarray(flat, dtype=np.float32).reshape(-1)
    return {name: flat[off:off + int(np.prod(shape))].reshape(shape).copy()
            for name, (off, shape) in ffi.MLP_LAYOUT.items()}


def harvest(sim, steps: int = 20, dt: float = 0.0, target_mode: int = ffi.SPH_TARGET_SOLVED):
    """Run `steps` KDK steps and collect one (features, target) row per
    particle and step (target_mode: ffi.SPH_TARGET_SOLVED or _CENTRED).
    Returns device tensors feat [steps*n, 8] and target [steps*n] (float32)."""
    n = sim.n
    feat = torch.zeros((steps * n, ffi.SPH_MLP_NFEAT), dtype=torch.float32, device=sim.device)
    target = torch.zeros(steps * n, dtype=torch.float32, device=sim.device)
    try:
        for k in range(steps):
            sim.set_harvest(feat[k * n:(k + 1) * n], target[k * n:(k + 1) * n], target_mode)
            sim.step(dt)
    finally:
        sim.set_harvest(None, None)
    return feat, target


def train(sim, feat: torch.Tensor, target: torch.Tensor, seed: int, epochs: int = 4,
          batch: int = 8192, lr: float = 1e-3, init: dict | None = None):
    """Fit the standardisation on the rows, initialise the weights (Xavier
    uniform from `seed` unless `init` is given) and run the epoch loop on the
    device.  Returns (weights dict, norm12, per-batch losses)."""
    n = int(feat.shape[0])
    w0 = init if init is not None else inputs.mlp_init(seed)
    sim.set_mlp(w0)
    ffi.sph_mlp_fit_norm(sim.ctx, feat.data_ptr(), n)
    flat0, norm = sim.get_mlp()
    sim.set_mlp(flat0, norm)   # clears the Adam state
    # row order: a seeded permutation drawn on the device (hundreds of
    # millions of rows at the full workloads)
    gen = torch.Generator(device=sim.device).manual_seed(seed)
    order = torch.randperm(n, generator=gen, device=sim.device, dtype=torch.int32)
    nb = (n + batch - 1) // batch
    loss = torch.zeros(max(epochs * nb, 1), dtype=torch.float32, device=sim.device)
    ffi.sph_mlp_train(sim.ctx, feat.data_ptr(), target.data_ptr(), order.data_ptr(), n, batch,
                      epochs, lr, loss.data_ptr())
    flat, norm = sim.get_mlp()
    return unpack_params(flat), norm, loss[: epochs * nb].cpu().numpy()


def evaluate_model(sim, feat: torch.Tensor, target: torch.Tensor) -> float:
    """Mean squared error of the current weights on (feat, target) rows."""
    n = int(feat.shape[0])
    grad = torch.zeros(ffi.SPH_MLP_NPARAM + 1, dtype=torch.float32, device=sim.device)
    ffi.sph_mlp_backward(sim.ctx, feat.data_ptr(), target.data_ptr(), None, 0, n,
                         grad.data_ptr())
    return float(grad[-1].item())
