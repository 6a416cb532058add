"""The C ABI library loads and exports every symbol the public header
declares (no compute calls: this runs without a GPU), and host-side
parameter validation behaves as documented."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADERS = [os.path.join(ROOT, "include", f) for f in sorted(os.listdir(os.path.join(ROOT, "include")))
           if f.endswith(".h")]


def _declared():
    names = set()
    for h in HEADERS:
        txt = open(h).read()
        txt = re.sub(r"/\*.*?\*/", "", txt, flags=re.S)
        for m in re.finditer(r"\b(sph_\w+)\s*\(", txt):
            names.add(m.group(1))
    return sorted(names)


@pytest.fixture(scope="module")
def lib():
    from paper_1905_03344_amd import ffi
    if not os.path.exists(ffi.LIB_PATH):
        from paper_1905_03344_amd import build
        build.build()
    return ffi.lib()


def test_every_declared_symbol_is_exported(lib):
    names = _declared()
    assert len(names) >= 15
    for n in names:
        assert hasattr(lib, n), n


def test_binding_covers_every_declared_symbol(lib):
    from paper_1905_03344_amd import ffi
    assert set(_declared()) <= set(ffi.exported_symbols())


def test_params_validation(lib):
    from paper_1905_03344_amd import ffi
    p = ffi.default_params()
    assert p.n_target == 100 and p.n_tol == 5 and p.list_stride == 128
    assert abs(p.gamma - 5.0 / 3.0) < 1e-15 and p.av_alpha == 1.0 and p.av_beta == 2.0
    p.n_max = 1000
    ctx = ffi.sph_create(p)
    assert ctx
    ffi.sph_destroy(ctx)
    bad = ffi.default_params()
    bad.max_level = 9
    with pytest.raises(ffi.SphError) as e:
        ffi.sph_create(bad)
    assert e.value.code == ffi.SPH_EINVAL and "max_level" in str(e.value)
    bad = ffi.default_params()
    bad.periodic[2] = 1
    with pytest.raises(ffi.SphError):
        ffi.sph_create(bad)
    assert p.walk_prefilter == ffi.SPH_PREFILTER_MATRIX
    bad = ffi.default_params()
    bad.walk_prefilter = 2
    with pytest.raises(ffi.SphError) as e:
        ffi.sph_create(bad)
    assert "walk_prefilter" in str(e.value)
    assert p.grad_h == 0
    for gh, prec in ((2, ffi.SPH_FP64), (-1, ffi.SPH_MIXED)):
        bad = ffi.default_params()
        bad.grad_h = gh
        bad.precision = prec
        with pytest.raises(ffi.SphError) as e:
            ffi.sph_create(bad)
        assert "grad_h" in str(e.value)
    assert p.gradients == ffi.SPH_GRADIENTS_KERNEL
    assert p.walk_defer_group == 0
    bad = ffi.default_params()
    bad.walk_defer_group = 65
    with pytest.raises(ffi.SphError) as e:
        ffi.sph_create(bad)
    assert "walk_defer_group" in str(e.value)
    for gr, prec in ((2, ffi.SPH_FP64), (-1, ffi.SPH_MIXED)):
        bad = ffi.default_params()
        bad.gradients = gr
        bad.precision = prec
        with pytest.raises(ffi.SphError) as e:
            ffi.sph_create(bad)
        assert "gradients" in str(e.value) or "IAD" in str(e.value)
    assert p.learned_try_shell == ffi.SPH_TRY_SHELL_AUTO
    for v in (-1, 3):
        bad = ffi.default_params()
        bad.learned_try_shell = v
        with pytest.raises(ffi.SphError) as e:
            ffi.sph_create(bad)
        assert "learned_try_shell" in str(e.value)


def test_workspace_size_grows_with_n(lib):
    from paper_1905_03344_amd import ffi
    p = ffi.default_params()
    p.n_max = 1000
    a = ffi.sph_workspace_size(p)
    p.n_max = 1000000
    b = ffi.sph_workspace_size(p)
    assert b > a > 0


def test_unbound_context_rejects_calls(lib):
    from paper_1905_03344_amd import ffi
    p = ffi.default_params()
    p.n_max = 10
    ctx = ffi.sph_create(p)
    s = ffi.sph_particles()
    rc = lib.sph_build_cells(ctx, ctypes.byref(s))
    assert rc == ffi.SPH_ENOMEM
    assert b"workspace" in lib.sph_last_error(ctx)
    ffi.sph_destroy(ctx)


def test_missing_library_fails_loudly():
    """Without the built library the binding raises; there is no CPU path."""
    import subprocess
    import sys
    code = ("from paper_1905_03344_amd import ffi\n"
            "ffi.LIB_PATH = '/nonexistent/libsph.so'\n"
            "ffi._lib = None\n"
            "try:\n"
            "    ffi.lib()\n"
            "except ImportError as e:\n"
            "    print('raised', e)\n")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-c", code], capture_output=True, text=True, cwd=root,
                         timeout=120)
    assert out.returncode == 0 and out.stdout.startswith("raised"), out.stdout + out.stderr
