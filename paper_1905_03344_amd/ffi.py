"""ctypes binding of libsph (include/sph.h): structures and the entry points,
under the same names.  Argument marshalling only -- every step of the path
runs in the library's HIP kernels.  Importing this module loads the in-tree
``libsph.so`` and fails loudly if it is missing."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libsph.so")

SPH_OK = 0
SPH_EINVAL = -1
SPH_ENOMEM = -2
SPH_ECAPACITY = -3
SPH_EHIP = -4
SPH_ENONFINITE = -5
SPH_WNOCONV = 1

SPH_INTEGRATOR_KDK = 0
SPH_INTEGRATOR_AB2 = 1
SPH_GRADIENTS_KERNEL = 0
SPH_GRADIENTS_IAD = 1
SPH_VOLUMES_STANDARD = 0
SPH_VOLUMES_GENERALIZED = 1
SPH_KERNEL_M4 = 0
SPH_KERNEL_WENDLAND = 1
SPH_KERNEL_SINC5 = 2
SPH_FP64 = 0
SPH_MIXED = 1
SPH_PREFILTER_NONE = 0
SPH_PREFILTER_MATRIX = 1
SPH_WALK_AUTO = 0
SPH_WALK_SHELL_FIRST = 1
SPH_WALK_WORKLIST = 2
SPH_TRY_SHELL_AUTO = 0
SPH_TRY_SHELL_NEVER = 1
SPH_TRY_SHELL_ALWAYS = 2
SPH_H_PLAIN = 0
SPH_H_LEARNED = 1
SPH_FLAG_NOCONV = 1
SPH_FLAG_LEARNED = 2

_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_D = ctypes.c_double


class sph_params(ctypes.Structure):
    _fields_ = [("n_max", _I64), ("list_stride", _I32), ("integrator", _I32),
                ("extra_slots", _I32), ("walk_prefilter", _I32), ("periodic", _I32 * 3), ("kernel", _I32),
                ("box_lo", _D * 3), ("box_hi", _D * 3), ("n_target", _I32), ("n_tol", _I32),
                ("h_max_iter", _I32), ("precision", _I32), ("gamma", _D), ("av_alpha", _D),
                ("av_beta", _D), ("av_eta2", _D), ("cfl", _D), ("h_mode", _I32),
                ("check_finite", _I32), ("max_level", _I32), ("search_div", _I32),
                ("grad_h", _I32), ("gradients", _I32), ("walk_defer_group", _I32),
                ("volumes", _I32), ("walk_strategy", _I32), ("gve_exponent", _D),
                ("learned_try_shell", _I32), ("pad1", _I32)]


CARRIED_F64 = ("x", "y", "z", "vx", "vy", "vz", "m", "h", "u", "ax", "ay", "az", "du", "rho",
               "divv")
CARRIED_I32 = ("nc", "id")
SINGLE_F64 = ("pvx", "pvy", "pvz", "pu", "p", "c")


class sph_particles(ctypes.Structure):
    _fields_ = ([("n", _I64), ("cur", _I32), ("pad0", _I32)]
                + [(f, _P * 2) for f in CARRIED_F64]
                + [(f, _P * 2) for f in CARRIED_I32]
                + [(f, _P) for f in SINGLE_F64]
                + [("flags", _P), ("key", _P), ("perm", _P)])


class sph_nlist(ctypes.Structure):
    _fields_ = [("idx", _P), ("stride", _I64), ("ecnt", _P), ("eidx", _P)]


class sph_stats(ctypes.Structure):
    _fields_ = [("nonconverged", _I64), ("list_overflow", _I64), ("extra_total", _I64),
                ("extra_overflow", _I64), ("nonfinite", _I64), ("h_counts", _I64),
                ("learned_accepted", _I64), ("learned_fallback", _I64), ("candidates", _I64),
                ("dt", _D), ("candidates_first", _I64), ("iad_singular", _I64),
                ("csr_overflow", _I64)]

    def as_dict(self):
        return {k: getattr(self, k) for k, _ in self._fields_}


class SphError(RuntimeError):
    def __init__(self, code, msg):
        super().__init__(f"libsph error {code}: {msg}")
        self.code = code


_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "sph_default_params": (None, [ctypes.POINTER(sph_params)]),
    "sph_create": (ctypes.c_int, [ctypes.POINTER(sph_params), ctypes.POINTER(_P)]),
    "sph_destroy": (None, [_P]),
    "sph_params_error": (ctypes.c_char_p, []),
    "sph_workspace_size": (ctypes.c_int, [ctypes.POINTER(sph_params), ctypes.POINTER(ctypes.c_size_t)]),
    "sph_bind": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "sph_build_cells": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles)]),
    "sph_find_neighbors": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist)]),
    "sph_density": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist)]),
    "sph_eos": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles)]),
    "sph_momentum_energy": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist), _P]),
    "sph_evaluate": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist), _P]),
    "sph_step": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist), _D, _P]),
    "sph_conservation": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), _P]),
    "sph_interaction_csr": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), ctypes.POINTER(sph_nlist), _P, _P, _I64]),
    "sph_conservation_noalloc": (ctypes.c_int, [ctypes.POINTER(sph_particles), _P, _P]),
    "sph_sync": (ctypes.c_int, [_P, ctypes.POINTER(sph_stats)]),
    "sph_last_error": (ctypes.c_char_p, [_P]),
    "sph_copy_internal": (ctypes.c_int, [_P, ctypes.c_int, _P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_size_t)]),
    "sph_timing": (ctypes.c_int, [_P, ctypes.c_int]),
    "sph_timing_read": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64), ctypes.c_int]),
    "sph_mlp_set_weights": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_D)]),
    "sph_mlp_get_weights": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_float), ctypes.POINTER(_D)]),
    "sph_mlp_fit_norm": (ctypes.c_int, [_P, _P, _I64]),
    "sph_get_features": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), _P, _P]),
    "sph_get_omega": (ctypes.c_int, [_P, ctypes.POINTER(sph_particles), _P]),
    "sph_set_harvest": (ctypes.c_int, [_P, _P, _P, _I32]),
    "sph_mlp_forward": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P]),
    "sph_mlp_backward": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I64, _P]),
    "sph_mlp_adam_step": (ctypes.c_int, [_P, _P, _D, _D, _D, _D, _I32]),
    "sph_mlp_train": (ctypes.c_int, [_P, _P, _P, _P, _I64, _I32, _I32, _D, _P]),
}

SPH_MLP_NPARAM = 4673
SPH_MLP_NFEAT = 8
# parameter layout: name -> (offset, shape)
MLP_LAYOUT = {"W1": (0, (64, 6)), "b1": (384, (64,)), "W2": (448, (64, 64)),
              "b2": (4544, (64,)), "W3": (4608, (1, 64)), "b3": (4672, (1,))}

STAGES = ("cells", "hsolve", "extra", "density", "eos", "forces", "integrate", "mlp", "hwalk")

# entry points of the learned / mixed forms, bound when present
_OPTIONAL = {}


def lib():
    """Load libsph.so (in-tree).  Raises if it has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1905_03344_amd.build` (hipcc, gfx950)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in {**_SIGS, **_OPTIONAL}.items():
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def exported_symbols():
    return list(_SIGS) + list(_OPTIONAL)


def register_optional(name, res, args):
    _OPTIONAL[name] = (res, args)
    if _lib is not None:
        fn = getattr(_lib, name)
        fn.restype = res
        fn.argtypes = args


def check(code, ctx=None, allow=(SPH_OK,)):
    if code in allow:
        return code
    msg = ""
    if ctx is not None:
        raw = lib().sph_last_error(ctx)
        msg = raw.decode() if raw else ""
    elif code == SPH_EINVAL:
        raw = lib().sph_params_error()
        msg = raw.decode() if raw else ""
    raise SphError(code, msg)


def default_params() -> sph_params:
    p = sph_params()
    lib().sph_default_params(ctypes.byref(p))
    return p


# thin wrappers with the C names ------------------------------------------------

def sph_create(p: sph_params):
    h = _P()
    check(lib().sph_create(ctypes.byref(p), ctypes.byref(h)))
    return h


def sph_destroy(ctx):
    lib().sph_destroy(ctx)


def sph_workspace_size(p: sph_params) -> int:
    n = ctypes.c_size_t()
    check(lib().sph_workspace_size(ctypes.byref(p), ctypes.byref(n)))
    return n.value


def sph_bind(ctx, ws_ptr: int, nbytes: int, stream: int):
    check(lib().sph_bind(ctx, ws_ptr, nbytes, stream), ctx)


def sph_build_cells(ctx, s: sph_particles):
    check(lib().sph_build_cells(ctx, ctypes.byref(s)), ctx)


def sph_find_neighbors(ctx, s, nl):
    check(lib().sph_find_neighbors(ctx, ctypes.byref(s), ctypes.byref(nl)), ctx)


def sph_density(ctx, s, nl):
    check(lib().sph_density(ctx, ctypes.byref(s), ctypes.byref(nl)), ctx)


def sph_eos(ctx, s):
    check(lib().sph_eos(ctx, ctypes.byref(s)), ctx)


def sph_momentum_energy(ctx, s, nl, d_dt: int):
    check(lib().sph_momentum_energy(ctx, ctypes.byref(s), ctypes.byref(nl), d_dt), ctx)


def sph_evaluate(ctx, s, nl, d_dt: int):
    check(lib().sph_evaluate(ctx, ctypes.byref(s), ctypes.byref(nl), d_dt), ctx)


def sph_step(ctx, s, nl, dt: float, d_dt: int):
    check(lib().sph_step(ctx, ctypes.byref(s), ctypes.byref(nl), float(dt), d_dt), ctx)


def sph_interaction_csr(ctx, s, nl, d_off: int, d_idx: int, capacity: int):
    check(lib().sph_interaction_csr(ctx, ctypes.byref(s), ctypes.byref(nl), d_off, d_idx,
                                    int(capacity)), ctx)


def sph_conservation(ctx, s, d_out7: int):
    check(lib().sph_conservation(ctx, ctypes.byref(s), d_out7), ctx)


def sph_conservation_noalloc(s, d_out7: int, stream: int):
    """The allocation-free variant (no context; stream is a hipStream_t)."""
    code = lib().sph_conservation_noalloc(ctypes.byref(s), d_out7, stream)
    if code != SPH_OK:
        raise SphError(code, "sph_conservation_noalloc: " +
                       ("invalid argument" if code == SPH_EINVAL else "HIP runtime error"))


def sph_sync(ctx, allow=(SPH_OK, SPH_WNOCONV)):
    st = sph_stats()
    code = lib().sph_sync(ctx, ctypes.byref(st))
    check(code, ctx, allow)
    return code, st


def sph_copy_internal(ctx, which: int, dst: int, nbytes: int) -> int:
    need = ctypes.c_size_t()
    check(lib().sph_copy_internal(ctx, which, dst, nbytes, ctypes.byref(need)), ctx)
    return need.value


def sph_timing(ctx, enable: bool):
    check(lib().sph_timing(ctx, int(bool(enable))), ctx)


def sph_timing_read(ctx):
    """{stage: (total_ms, intervals)} since timing was enabled."""
    ms = (ctypes.c_double * len(STAGES))()
    cnt = (_I64 * len(STAGES))()
    check(lib().sph_timing_read(ctx, ms, cnt, len(STAGES)), ctx)
    return {s: (ms[k], cnt[k]) for k, s in enumerate(STAGES)}


# learned smoothing length ---------------------------------------------------

def _f32buf(a):
    import numpy as np
    a = np.ascontiguousarray(a, dtype=np.float32)
    return a, a.ctypes.data_as(ctypes.POINTER(ctypes.c_float))


def sph_mlp_set_weights(ctx, params, norm12=None):
    """params: SPH_MLP_NPARAM floats (host); norm12: mean[6] + std[6] or None."""
    import numpy as np
    a, pa = _f32buf(params)
    if a.size != SPH_MLP_NPARAM:
        raise ValueError(f"expected {SPH_MLP_NPARAM} parameters, got {a.size}")
    pn = None
    if norm12 is not None:
        nb = np.ascontiguousarray(norm12, dtype=np.float64)
        if nb.size != 12:
            raise ValueError("norm12 must hold 12 values")
        pn = nb.ctypes.data_as(ctypes.POINTER(_D))
    check(lib().sph_mlp_set_weights(ctx, pa, pn), ctx)


def sph_mlp_get_weights(ctx):
    import numpy as np
    params = np.zeros(SPH_MLP_NPARAM, dtype=np.float32)
    norm = np.zeros(12, dtype=np.float64)
    check(lib().sph_mlp_get_weights(ctx, params.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                    norm.ctypes.data_as(ctypes.POINTER(_D))), ctx)
    return params, norm


def sph_mlp_fit_norm(ctx, d_feat: int, n: int):
    check(lib().sph_mlp_fit_norm(ctx, d_feat, n), ctx)


def sph_get_features(ctx, s, d_dt: int, d_feat: int):
    check(lib().sph_get_features(ctx, ctypes.byref(s), d_dt, d_feat), ctx)


def sph_get_omega(ctx, s, d_omega: int):
    check(lib().sph_get_omega(ctx, ctypes.byref(s), d_omega), ctx)


SPH_TARGET_SOLVED = 0
SPH_TARGET_CENTRED = 1


def sph_set_harvest(ctx, d_feat: int | None, d_target: int | None,
                    target_mode: int = SPH_TARGET_SOLVED):
    check(lib().sph_set_harvest(ctx, d_feat, d_target, target_mode), ctx)


def sph_mlp_forward(ctx, d_feat: int, n: int, d_y: int, d_h1: int | None = None,
                    d_h2: int | None = None):
    check(lib().sph_mlp_forward(ctx, d_feat, n, d_y, d_h1, d_h2), ctx)


def sph_mlp_backward(ctx, d_feat: int, d_target: int, d_rows: int | None, row0: int, n: int,
                     d_grad: int):
    check(lib().sph_mlp_backward(ctx, d_feat, d_target, d_rows, row0, n, d_grad), ctx)


def sph_mlp_adam_step(ctx, d_grad: int, lr: float, beta1: float, beta2: float, eps: float,
                      t: int):
    check(lib().sph_mlp_adam_step(ctx, d_grad, lr, beta1, beta2, eps, t), ctx)


def sph_mlp_train(ctx, d_feat: int, d_target: int, d_order: int | None, n: int, batch: int,
                  epochs: int, lr: float, d_loss: int | None):
    check(lib().sph_mlp_train(ctx, d_feat, d_target, d_order, n, batch, epochs, lr, d_loss), ctx)
