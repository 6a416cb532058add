"""Device-resident particle state for libsph: torch tensors provide the
memory and the stream, the library's kernels do all the work.

    sim = Simulation(ic, params)          # ic: inputs.ParticleSet
    sim.evaluate()                        # forces at t = 0
    for _ in range(steps): sim.step()     # KDK steps at the Courant dt
"""
from __future__ import annotations

import ctypes
import math

import numpy as np
import torch

from . import ffi


def choose_max_level(n: int, bbox_extent: float, h_min: float, search_div: int = 1) -> int:
    """Finest cell level the table needs so that search cells can be about
    2 h_min / search_div wide (between 1 and 8)."""
    if h_min <= 0 or bbox_extent <= 0:
        return 1
    want = bbox_extent * search_div / (2.0 * h_min)
    lvl = int(math.floor(math.log2(max(want, 1.0))))
    return max(1, min(8, lvl + 1))


class Simulation:
    def __init__(self, ic, params: ffi.sph_params | None = None, device="cuda", n_max=None,
                 list_stride=128, extra_per_particle=48, max_level=None, search_div=2,
                 precision=ffi.SPH_FP64, check_finite=False, h_mode=ffi.SPH_H_PLAIN,
                 walk_prefilter=None, kernel=None, integrator=None, grad_h=False,
                 gradients=None, walk_defer_group=None, volumes=None, gve_exponent=None,
                 walk_strategy=None, learned_try_shell=None):
        """Allocate the state and the workspace for ic and bind a context.

        precision: ffi.SPH_FP64 or ffi.SPH_MIXED; h_mode: ffi.SPH_H_PLAIN or
        ffi.SPH_H_LEARNED (weights via set_mlp); kernel: ffi.SPH_KERNEL_*;
        integrator: ffi.SPH_INTEGRATOR_KDK or _AB2; grad_h: grad-h correction
        terms; gradients: ffi.SPH_GRADIENTS_KERNEL or _IAD; volumes:
        ffi.SPH_VOLUMES_STANDARD or _GENERALIZED (weights (m/rho)^gve_exponent); walk_prefilter:
        ffi.SPH_PREFILTER_MATRIX or _NONE; walk_strategy: ffi.SPH_WALK_*; walk_defer_group: first-round
        sub-groups up to this size go to the per-particle tail; learned_try_shell:
        ffi.SPH_TRY_SHELL_* (the last three speed only).
        None keeps the library default.
        list_stride and extra_per_particle are the capacities of the gather
        and complement rows; max_level None picks the cell level from the
        extent and the smallest h."""
        self.device = torch.device(device)
        n = ic.n
        self.n = n
        p = params if params is not None else ffi.default_params()
        p.n_max = int(n_max or n)
        p.list_stride = int(list_stride)
        p.extra_slots = int(extra_per_particle)
        for d in range(3):
            p.periodic[d] = int(ic.periodic[d])
            p.box_lo[d] = float(ic.box_lo[d])
            p.box_hi[d] = float(ic.box_hi[d])
        if max_level is None:
            if n > 0:
                ext = max(float(np.ptp(ic.x)), float(np.ptp(ic.y)), float(np.ptp(ic.z)), 1e-300)
                max_level = choose_max_level(n, ext, float(np.min(ic.h)) * 0.7, search_div)
            else:
                max_level = 1
        p.max_level = int(max_level)
        p.search_div = int(search_div)
        if walk_prefilter is not None:
            p.walk_prefilter = int(walk_prefilter)
        if kernel is not None:
            p.kernel = int(kernel)
        if integrator is not None:
            p.integrator = int(integrator)
        p.grad_h = int(bool(grad_h))
        if gradients is not None:
            p.gradients = int(gradients)
        if walk_defer_group is not None:
            p.walk_defer_group = int(walk_defer_group)
        if volumes is not None:
            p.volumes = int(volumes)
        if walk_strategy is not None:
            p.walk_strategy = int(walk_strategy)
        if learned_try_shell is not None:
            p.learned_try_shell = int(learned_try_shell)
        if gve_exponent is not None:
            p.gve_exponent = float(gve_exponent)
        p.precision = int(precision)
        p.check_finite = int(bool(check_finite))
        p.h_mode = int(h_mode)
        self.params = p
        self.ctx = ffi.sph_create(p)
        dev = self.device
        f64 = dict(dtype=torch.float64, device=dev)
        i32 = dict(dtype=torch.int32, device=dev)
        self.t = {}
        for f in ffi.CARRIED_F64:
            self.t[f] = [torch.zeros(n, **f64), torch.zeros(n, **f64)]
        for f in ffi.CARRIED_I32:
            self.t[f] = [torch.zeros(n, **i32), torch.zeros(n, **i32)]
        for f in ffi.SINGLE_F64:
            self.t[f] = torch.zeros(n, **f64)
        self.t["flags"] = torch.zeros(n, dtype=torch.uint8, device=dev)
        self.t["key"] = torch.zeros(n, **i32)   # uint32 bits in an int32 tensor
        self.t["perm"] = torch.zeros(n, **i32)
        arrays = ic.arrays()
        for f in ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u"):
            self.t[f][0].copy_(torch.from_numpy(np.ascontiguousarray(arrays[f], dtype=np.float64)))
        self.t["id"][0].copy_(torch.arange(n, dtype=torch.int32))
        # neighbour lists
        self.stride = max(64, ((n + 63) // 64) * 64)
        self.nl_idx = torch.zeros(p.list_stride * self.stride, **i32)
        self.nl_ecnt = torch.zeros(self.stride, **i32)
        self.nl_eidx = torch.zeros(p.extra_slots * self.stride, **i32)
        self.d_dt = torch.zeros(1, **f64)
        self.cons = torch.zeros(8, **f64)
        # workspace
        self.ws_bytes = ffi.sph_workspace_size(p)
        self.ws = torch.empty(self.ws_bytes, dtype=torch.uint8, device=dev)
        self.stream = torch.cuda.current_stream(dev)
        ffi.sph_bind(self.ctx, self.ws.data_ptr(), self.ws_bytes, self.stream.cuda_stream)
        self.s = ffi.sph_particles()
        self.s.n = n
        self.s.cur = 0
        self._fill_ptrs()
        self.nl = ffi.sph_nlist()
        self.nl.idx = self.nl_idx.data_ptr()
        self.nl.stride = self.stride
        self.nl.ecnt = self.nl_ecnt.data_ptr()
        self.nl.eidx = self.nl_eidx.data_ptr()
        self.time = 0.0

    def _fill_ptrs(self):
        s = self.s
        for f in ffi.CARRIED_F64 + ffi.CARRIED_I32:
            arr = getattr(s, f)
            arr[0] = self.t[f][0].data_ptr()
            arr[1] = self.t[f][1].data_ptr()
        for f in ffi.SINGLE_F64 + ("flags", "key", "perm"):
            setattr(s, f, self.t[f].data_ptr())

    def __del__(self):
        try:
            if getattr(self, "ctx", None):
                ffi.sph_destroy(self.ctx)
                self.ctx = None
        except Exception:
            pass

    # --- field access -------------------------------------------------------
    @property
    def cur(self):
        return self.s.cur

    def field(self, name):
        """Current buffer of a carried field, or a single buffer."""
        v = self.t[name]
        return v[self.s.cur] if isinstance(v, list) else v

    def numpy(self, name):
        a = self.field(name).cpu().numpy()
        if name == "key":
            a = a.view(np.uint32)
        return a

    def omega(self):
        """Grad-h factors of the last density evaluation (grad_h contexts)."""
        out = torch.empty(self.n, dtype=torch.float64, device=self.device)
        ffi.sph_get_omega(self.ctx, self.s, out.data_ptr())
        self.sync()
        return out.cpu().numpy()

    def set_field(self, name, values):
        self.field(name).copy_(torch.as_tensor(np.ascontiguousarray(values)).to(self.device))

    # --- stages -------------------------------------------------------------
    def build_cells(self):
        ffi.sph_build_cells(self.ctx, self.s)

    def find_neighbors(self):
        ffi.sph_find_neighbors(self.ctx, self.s, self.nl)

    def density(self):
        ffi.sph_density(self.ctx, self.s, self.nl)

    def eos(self):
        ffi.sph_eos(self.ctx, self.s)

    def momentum_energy(self):
        ffi.sph_momentum_energy(self.ctx, self.s, self.nl, self.d_dt.data_ptr())

    def evaluate(self):
        ffi.sph_evaluate(self.ctx, self.s, self.nl, self.d_dt.data_ptr())

    def step(self, dt: float = 0.0):
        ffi.sph_step(self.ctx, self.s, self.nl, float(dt), self.d_dt.data_ptr())

    def conservation(self):
        ffi.sph_conservation(self.ctx, self.s, self.cons.data_ptr())
        return self.cons[:7].cpu().numpy().copy()

    def sync(self, allow=(ffi.SPH_OK, ffi.SPH_WNOCONV)):
        return ffi.sph_sync(self.ctx, allow)

    def dt(self):
        return float(self.d_dt.item())

    def copy_pred_from_state(self):
        """pv = v, pu = u (what sph_evaluate does before the force stages)."""
        for a, b in (("pvx", "vx"), ("pvy", "vy"), ("pvz", "vz"), ("pu", "u")):
            self.t[a].copy_(self.field(b))

    # --- learned smoothing length ---------------------------------------------
    def set_mlp(self, params, norm12=None):
        """params: flat SPH_MLP_NPARAM floats or a dict W1, b1, W2, b2, W3, b3."""
        from .learned import pack_params
        flat = pack_params(params) if isinstance(params, dict) else params
        ffi.sph_mlp_set_weights(self.ctx, flat, norm12)

    def get_mlp(self):
        """(flat FP32 parameters, norm12) from the device."""
        return ffi.sph_mlp_get_weights(self.ctx)

    def features(self):
        """Feature rows [n, 8] of the current state (dt of the last step)."""
        out = torch.zeros((max(self.n, 1), ffi.SPH_MLP_NFEAT), dtype=torch.float32,
                          device=self.device)
        ffi.sph_get_features(self.ctx, self.s, self.d_dt.data_ptr(), out.data_ptr())
        return out[: self.n]

    def set_harvest(self, feat: torch.Tensor | None, target: torch.Tensor | None,
                    target_mode: int = ffi.SPH_TARGET_SOLVED):
        """Every later step writes its (features, target) rows into these
        device tensors ([>= n, 8] float32 and [>= n] float32); None stops."""
        if feat is None:
            ffi.sph_set_harvest(self.ctx, None, None)
            return
        assert feat.dtype == torch.float32 and target.dtype == torch.float32
        assert feat.is_contiguous() and target.is_contiguous()
        assert feat.shape[0] >= self.n and feat.shape[1] == ffi.SPH_MLP_NFEAT
        assert target.shape[0] >= self.n
        ffi.sph_set_harvest(self.ctx, feat.data_ptr(), target.data_ptr(), target_mode)

    # --- tables and lists for tests ------------------------------------------
    def cell_table(self):
        need = ffi.sph_copy_internal(self.ctx, 0, 0, 0)
        out = torch.zeros(need // 4, dtype=torch.int32, device=self.device)
        ffi.sph_copy_internal(self.ctx, 0, out.data_ptr(), need)
        return out.cpu().numpy()

    def bbox(self):
        out = torch.zeros(6, dtype=torch.float64, device=self.device)
        ffi.sph_copy_internal(self.ctx, 1, out.data_ptr(), 48)
        return out.cpu().numpy()

    def gather_lists(self):
        """(nc, L) with L a list of per-particle int32 arrays in stored order."""
        n = self.n
        nc = self.numpy("nc")
        K = self.params.list_stride
        idx = self.nl_idx.view(self.stride, K)[:n].cpu().numpy().T
        return nc, [idx[:min(int(nc[i]), K), i] for i in range(n)]

    def gather_dense(self):
        """(nc, idx[K, n]) numpy view of the gather sets."""
        n = self.n
        K = self.params.list_stride
        return self.numpy("nc"), self.nl_idx.view(self.stride, K)[:n].cpu().numpy().T

    def extra_lists(self):
        """(eoff, eidx): the complement rows as CSR with ascending rows."""
        n = self.n
        ke = self.params.extra_slots
        ecnt = np.minimum(self.nl_ecnt[:n].cpu().numpy(), ke)
        e = self.nl_eidx.view(self.stride, ke)[:n].cpu().numpy().T
        mask = np.arange(ke)[:, None] < ecnt[None, :]
        kk, ii = np.nonzero(mask)
        code = np.sort(ii.astype(np.int64) * max(n, 1) + e[kk, ii].astype(np.int64))
        eoff = np.concatenate([[0], np.cumsum(np.bincount(ii, minlength=n))]).astype(np.int64)
        return eoff, (code % max(n, 1)).astype(np.int32)

    def interaction_csr_device(self):
        """S_i = L_i U E_i as CSR with ascending rows, built by the library
        (sph_interaction_csr): (off int64[n+1], idx int32[total]) tensors."""
        off = torch.zeros(self.n + 1, dtype=torch.int64, device=self.device)
        ffi.sph_interaction_csr(self.ctx, self.s, self.nl, off.data_ptr(), 0, 0)
        self.sync(allow=(ffi.SPH_OK, ffi.SPH_WNOCONV, ffi.SPH_ECAPACITY))
        total = int(off[-1].item())
        idx = torch.zeros(max(total, 1), dtype=torch.int32, device=self.device)
        ffi.sph_interaction_csr(self.ctx, self.s, self.nl, off.data_ptr(), idx.data_ptr(), total)
        self.sync()
        return off, idx[:total]

    def interaction_csr(self):
        """S_i = L_i U E_i as CSR with ascending rows (for comparisons)."""
        nc, idx = self.gather_dense()
        eoff, eidx = self.extra_lists()
        n = self.n
        K = self.params.list_stride
        rows = []
        off = np.zeros(n + 1, dtype=np.int64)
        for i in range(n):
            r = np.concatenate([idx[:min(int(nc[i]), K), i], eidx[eoff[i]:eoff[i + 1]]])
            r.sort()
            rows.append(r)
            off[i + 1] = off[i] + len(r)
        return off, (np.concatenate(rows) if rows else np.zeros(0, np.int32))
