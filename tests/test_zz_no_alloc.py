"""The allocation-free conservation entry point against the one that uses
the bound workspace, through the C ABI: the same kernels and block count,
so the seven sums must agree bit for bit.  Two calls in a row, the second
with a smaller input, so the per-GPU scratch array is reused with fewer
partial blocks than the first call left in it."""
import numpy as np
import pytest

from paper_1905_03344_amd import inputs

pytestmark = pytest.mark.gpu


def _both(sim):
    import torch
    from paper_1905_03344_amd import ffi
    out = torch.full((8,), float("nan"), dtype=torch.float64, device=sim.device)
    ffi.sph_conservation_noalloc(sim.s, out.data_ptr(), sim.stream.cuda_stream)
    torch.cuda.synchronize()
    got = out[:7].cpu().numpy().copy()
    ref = sim.conservation()
    return got, ref


def test_noalloc_conservation_matches_workspace_variant():
    from paper_1905_03344_amd.state import Simulation
    # 343,000 particles: 1340 blocks of 256 would be needed, so the launch
    # strides 1024 blocks over the array (the scratch's maximum)
    big = Simulation(inputs.square_patch(70, 31))
    big.evaluate()
    big.step(0.0)
    got, ref = _both(big)
    assert np.all(np.isfinite(got))
    np.testing.assert_array_equal(got, ref)
    del big
    # second call: a smaller input (46 blocks), after a step so every sum is
    # non-trivial
    small = Simulation(inputs.clumpy(n_clumps=4, per_clump=2500, n_background=1700, seed=5),
                       extra_per_particle=96)
    small.evaluate()
    small.step(0.0)
    got, ref = _both(small)
    np.testing.assert_array_equal(got, ref)
    assert np.all(np.abs(got[3:6]) > 0)


def test_noalloc_conservation_rejects_bad_arguments():
    import torch
    from paper_1905_03344_amd import ffi
    from paper_1905_03344_amd.state import Simulation
    sim = Simulation(inputs.square_patch(8, 3))
    out = torch.zeros(8, dtype=torch.float64, device=sim.device)
    s = ffi.sph_particles()
    ctypes_copy = type(sim.s).from_buffer_copy(sim.s)
    ctypes_copy.cur = 2
    with pytest.raises(ffi.SphError) as e:
        ffi.sph_conservation_noalloc(ctypes_copy, out.data_ptr(), sim.stream.cuda_stream)
    assert e.value.code == ffi.SPH_EINVAL
    ctypes_copy = type(sim.s).from_buffer_copy(sim.s)
    ctypes_copy.n = -1
    with pytest.raises(ffi.SphError):
        ffi.sph_conservation_noalloc(ctypes_copy, out.data_ptr(), sim.stream.cuda_stream)
    with pytest.raises(ffi.SphError):
        ffi.sph_conservation_noalloc(sim.s, 0, sim.stream.cuda_stream)
    del s
