"""Pins for the oracle's cell keys, sort, cell tables, neighbour counts, lists
and smoothing-length iteration, against independent brute-force code."""
import itertools

import numpy as np
import pytest

import oracle as O
from paper_1905_03344_amd import inputs


def _spread_bits(v):
    # independent Morton spreading with magic masks (not a bit loop)
    v = v.astype(np.uint64) & np.uint64(0x3FF)
    v = (v | (v << np.uint64(16))) & np.uint64(0x030000FF)
    v = (v | (v << np.uint64(8))) & np.uint64(0x0300F00F)
    v = (v | (v << np.uint64(4))) & np.uint64(0x030C30C3)
    v = (v | (v << np.uint64(2))) & np.uint64(0x09249249)
    return v


def _keys_numpy(ps, lo, hi):
    g = []
    for d, c in enumerate((ps.x, ps.y, ps.z)):
        L = hi[d] - lo[d]
        w = L / 1024.0
        t = (c - lo[d]) / w
        gi = np.clip(np.floor(t), 0, 1023).astype(np.int64)
        g.append(gi)
    k = _spread_bits(g[0]) | (_spread_bits(g[1]) << np.uint64(1)) | (_spread_bits(g[2]) << np.uint64(2))
    return k.astype(np.uint32)


def test_keys_match_independent_derivation():
    ps = inputs.square_patch(16, 7)
    lo, hi = O.bbox(ps.x, ps.y, ps.z, ps.periodic, ps.box_lo, ps.box_hi)
    assert tuple(lo) == (ps.x.min(), ps.y.min(), -0.5)
    assert tuple(hi) == (ps.x.max(), ps.y.max(), 0.5)
    k = O.cell_keys(ps.x, ps.y, ps.z, lo, hi)
    np.testing.assert_array_equal(k, _keys_numpy(ps, lo, hi))
    assert k.max() < (1 << 30)


def test_keys_clumpy_and_edges():
    ps = inputs.clumpy(n_clumps=4, per_clump=500, n_background=1000, seed=3)
    lo, hi = O.bbox(ps.x, ps.y, ps.z, ps.periodic, ps.box_lo, ps.box_hi)
    k = O.cell_keys(ps.x, ps.y, ps.z, lo, hi)
    np.testing.assert_array_equal(k, _keys_numpy(ps, lo, hi))
    # the maximum coordinate lands in cell 1023 of its dimension
    i = int(np.argmax(ps.x))
    assert (int(k[i]) & 0x09249249) == 0x09249249


def test_sort_is_stable_by_key():
    rng = np.random.default_rng(1)
    key = rng.integers(0, 50, size=5000).astype(np.uint32)   # many ties
    perm = O.sort_perm(key)
    np.testing.assert_array_equal(perm, np.argsort(key, kind="stable"))


@pytest.mark.parametrize("level", [0, 1, 2, 3])
def test_cell_start(level):
    ps = inputs.square_patch(12, 5)
    lo, hi = O.bbox(ps.x, ps.y, ps.z, ps.periodic, ps.box_lo, ps.box_hi)
    k = np.sort(O.cell_keys(ps.x, ps.y, ps.z, lo, hi))
    start = O.cell_start(k, level)
    cells = np.arange((1 << (3 * level)) + 1, dtype=np.uint64) << np.uint64(3 * (10 - level))
    np.testing.assert_array_equal(start, np.searchsorted(k.astype(np.uint64), cells, side="left"))
    assert start[-1] == len(k)


def _brute_r2(ps, periodic, box_lo, box_hi):
    pos = [ps.x, ps.y, ps.z]
    r2 = None
    comps = []
    for d in range(3):
        t = pos[d][None, :] - pos[d][:, None]    # x_j - x_i
        if periodic[d]:
            L = box_hi[d] - box_lo[d]
            t = np.where(t > 0.5 * L, t - L, np.where(t < -0.5 * L, t + L, t))
        comps.append(t)
    r2 = (comps[0] * comps[0] + comps[1] * comps[1]) + comps[2] * comps[2]
    return r2


def test_counts_brute_force_and_grid():
    ps = inputs.square_patch(11, 21)
    h = ps.h * (1.0 + 0.3 * inputs.uniform01(5, np.arange(ps.n)))
    r2 = _brute_r2(ps, ps.periodic, ps.box_lo, ps.box_hi)
    twoh = 2.0 * h
    expect = ((r2 < (twoh * twoh)[:, None]) & ~np.eye(ps.n, dtype=bool)).sum(1)
    for method in (0, 1):
        c = O.count(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, method)
        np.testing.assert_array_equal(c, expect)


def test_lists_symmetric_closure_brute_force():
    ps = inputs.clumpy(n_clumps=3, per_clump=400, n_background=300, seed=11)
    h = ps.h * 0.6
    r2 = _brute_r2(ps, ps.periodic, ps.box_lo, ps.box_hi)
    twoh = 2.0 * h
    L = (r2 < (twoh * twoh)[:, None]) & ~np.eye(ps.n, dtype=bool)
    S = L | L.T
    for method in (0, 1):
        off, idx = O.lists(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, method)
        assert off[-1] == S.sum()
        for i in range(ps.n):
            row = idx[off[i]:off[i + 1]]
            np.testing.assert_array_equal(row, np.nonzero(S[i])[0])


def test_lists_periodic_patch():
    ps = inputs.square_patch(10, 4)
    h = ps.h * (1.0 + 0.2 * inputs.uniform01(9, np.arange(ps.n)))
    r2 = _brute_r2(ps, ps.periodic, ps.box_lo, ps.box_hi)
    L = (r2 < ((2.0 * h) * (2.0 * h))[:, None]) & ~np.eye(ps.n, dtype=bool)
    S = L | L.T
    off, idx = O.lists(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, 1)
    dense = np.zeros_like(S)
    rows = np.repeat(np.arange(ps.n), np.diff(off))
    dense[rows, idx] = True
    np.testing.assert_array_equal(dense, S)
    assert np.all(np.diff(idx)[np.diff(rows) == 0] > 0)  # ascending rows


def _r3(nmax):
    # number of integer vectors with |k|^2 == n, by enumeration
    r = np.zeros(nmax + 1, dtype=int)
    m = int(np.ceil(np.sqrt(nmax))) + 1
    for a, b, c in itertools.product(range(-m, m + 1), repeat=3):
        s = a * a + b * b + c * c
        if s <= nmax:
            r[s] += 1
    return r


def test_lattice_shell_counts():
    # perfect periodic lattice: counts at 2h just above sqrt(n) s are the
    # cumulative lattice-vector numbers (self excluded)
    r3 = _r3(10)
    cum = np.cumsum(r3) - 1
    ps = inputs.perfect_lattice(12)
    s = ps.meta["s"]
    for nsq in (1, 2, 3, 4, 5, 6, 8, 9, 10):
        h = np.full(ps.n, 0.5 * np.sqrt(nsq) * s * (1 + 1e-9))
        c = O.count(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, 1)
        assert np.all(c == cum[nsq]), (nsq, c[:3], cum[nsq])
    assert list(cum[[1, 2, 3, 4, 5, 6, 8, 9, 10]]) == [6, 18, 26, 32, 56, 80, 92, 122, 146]


def test_hsolve_converges_in_band():
    ps = inputs.square_patch(14, 99)
    h, nc, flag, iters, nonconv = O.hsolve(ps.x, ps.y, ps.z, ps.h * 1.3, ps.periodic, ps.box_lo,
                                           ps.box_hi)
    assert nonconv == 0 and np.all(flag == 0)
    assert np.all(np.abs(nc - 100) <= 5)
    c = O.count(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, 0)
    np.testing.assert_array_equal(c, nc)
    assert iters.max() <= 32 and iters.min() >= 1


def test_hsolve_converged_input_takes_one_count():
    ps = inputs.square_patch(12, 3)
    h1, nc1, *_ = O.hsolve(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo, ps.box_hi)
    h2, nc2, flag, iters, _ = O.hsolve(ps.x, ps.y, ps.z, h1, ps.periodic, ps.box_lo, ps.box_hi)
    np.testing.assert_array_equal(h2, h1)
    assert np.all(iters == 1)


def test_hsolve_perfect_lattice_cannot_converge():
    # counts jump from 92 to 122 when 2h crosses 3s: no h gives 95..105.
    # spacing 1/16 makes every coordinate difference and square exact, so
    # each shell is exactly degenerate (with 1/12 rounding splits the shells
    # and bisection can land between their members)
    ps = inputs.perfect_lattice(16)
    h, nc, flag, iters, nonconv = O.hsolve(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo,
                                           ps.box_hi, max_iter=32)
    assert nonconv == ps.n and np.all(flag == 1)
    assert np.all(nc == 92)           # the best count by |N - 100|
    assert np.all(iters == 32)


def test_hsolve_clumpy():
    ps = inputs.clumpy(n_clumps=4, per_clump=1500, n_background=1500, seed=8)
    h, nc, flag, iters, nonconv = O.hsolve(ps.x, ps.y, ps.z, ps.h, ps.periodic, ps.box_lo,
                                           ps.box_hi)
    ok = flag == 0
    assert ok.mean() > 0.99
    assert np.all(np.abs(nc[ok] - 100) <= 5)
    c = O.count(ps.x, ps.y, ps.z, h, ps.periodic, ps.box_lo, ps.box_hi, 0)
    np.testing.assert_array_equal(c, nc)
    assert h.max() / h.min() > 4
