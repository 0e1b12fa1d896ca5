"""Pins for the oracle's PCDDT reading (CPU only).

The paper prunes the CDDT by casting from every state and dropping the zero
points no cast returns (Sec. IV-C), names it PCDDT, and reports it for static
maps.  The reading (cddt_ref.cpp, exact.py): the states are the free cells'
centres under every theta bin.  These tests tie it to what the paper and the
definition fix: casts from every state equal the unpruned structure and the
brute-force definition; nothing unused is kept (removing any kept point changes
some state's cast); the paper's co-linear example keeps exactly the two end
obstacles; the two independent oracles agree; the structure shrinks.
"""
import math

import numpy as np
import pytest

from oracle import exact
from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl


def _states(occ, n, jitter_rng=None):
    """Every free cell centre under every bin; with jitter_rng the angle moves inside the bin."""
    jj, ii = np.nonzero(occ == 0)
    x = np.repeat(ii.astype(np.float32) + np.float32(0.5), n)
    y = np.repeat(jj.astype(np.float32) + np.float32(0.5), n)
    k = np.tile(np.arange(n), ii.size)
    th = 2.0 * math.pi * k / n
    if jitter_rng is not None:
        th = th + jitter_rng.uniform(-0.45, 0.45, th.size) * (2.0 * math.pi / n)
    return x, y, th.astype(np.float32)


@pytest.mark.parametrize("seed", range(6))
def test_pruned_casts_equal_unpruned_at_every_state(seed):
    rng = wl.rng_for(951, seed)
    w, h = int(rng.integers(8, 70)), int(rng.integers(8, 70))
    occ = wl.random_map(rng, w, h, float(rng.uniform(0.05, 0.5)))
    n = int(rng.choice([2, 8, 36, 108]))
    full = bool(seed % 3 == 2)
    ex = oref.RefCDDT(occ, n, full_map=full)
    pr = oref.RefCDDT(occ, n, full_map=full, prune=True)
    for jit in (None, rng):
        x, y, th = _states(occ, n, jit)
        want = ex.cast(x, y, th, 10**6, threads=4)
        got = pr.cast(x, y, th, 10**6, threads=4)
        assert (got == want).all(), f"{(got != want).sum()} state casts differ"
        assert (got == ex.cast(x, y, th, 10**6, threads=4, brute=True)).all()   # Level-1 definition
    # pruning only removes: every pruned band is a subset of its unpruned band
    _, rl0, z0 = ex.export()
    _, rl1, z1 = pr.export()
    o0, o1 = np.concatenate([[0], np.cumsum(rl0)]), np.concatenate([[0], np.cumsum(rl1)])
    for b in np.nonzero(rl1)[0]:
        assert set(z1[o1[b]:o1[b + 1]].tolist()) <= set(z0[o0[b]:o0[b + 1]].tolist())
        assert (np.diff(z1[o1[b]:o1[b + 1]]) > 0).all()   # distinct, ascending


@pytest.mark.parametrize("seed", range(4))
def test_pruned_python_equals_cpp(seed):
    rng = wl.rng_for(952, seed)
    w, h = int(rng.integers(4, 16)), int(rng.integers(4, 16))
    occ = wl.random_map(rng, w, h, 0.3)
    n = int(rng.choice([4, 8, 16]))
    py = exact.PlainCDDT(occ, n, prune=True)
    cc = oref.RefCDDT(occ, n, prune=True)
    nr, rl, z = py.export()
    nr2, rl2, z2 = cc.export()
    assert (nr == nr2).all() and (rl == rl2).all() and (z == z2).all()


@pytest.mark.parametrize("seed", range(4))
def test_kept_points_are_exactly_the_brute_force_answers(seed):
    """Per band, the kept zero points are exactly the nearest zero points that the
    brute-force definition finds for the states landing there (nothing unused kept,
    nothing used dropped).  Ranges alone cannot show this: two kept points closer
    than one cell round to the same range."""
    rng = wl.rng_for(953, seed)
    occ = wl.random_map(rng, int(rng.integers(5, 14)), int(rng.integers(5, 14)), 0.35)
    n = int(rng.choice([4, 8, 16]))
    bf = exact.BruteForce(occ, n)
    tabs = exact.trig_table(n)
    want = {}
    x, y, th = _states(occ, n)
    for a, b_, t in zip(x, y, th):
        q = exact.prepare(occ, n, tabs, a, b_, t)
        assert q.valid
        z = bf.candidates(q)
        z = z[z > q.xq] if q.sigma > 0 else z[z < q.xq]
        if z.size:
            want.setdefault((q.s, q.r), set()).add(int(z.min() if q.sigma > 0 else z.max()))
    pr = oref.RefCDDT(occ, n, prune=True)
    nr, rl, zz = pr.export()
    c, s_, rmin, nrows, _ = pr.tables()
    o = np.concatenate([[0], np.cumsum(rl)])
    band = 0
    for sl in range(n // 2):
        for r in range(int(rmin[sl]), int(rmin[sl] + nrows[sl])):
            got = zz[o[band]:o[band + 1]].tolist()
            assert got == sorted(want.get((sl, r), set())), (sl, r)
            band += 1


def test_colinear_example_keeps_the_two_ends():
    """Sec. IV-C: a line of obstacles along x; at theta = 0 only its first and last cells survive."""
    occ = np.zeros((9, 20), np.uint8)
    j0, a, b = 4, 3, 15
    occ[j0, a:b + 1] = 1
    n = 8
    pr = oref.RefCDDT(occ, n, prune=True)
    nr, rl, z = pr.export()
    c, s, rmin, nrows, _ = pr.tables()
    assert c[0] == 1 << 30 and s[0] == 0            # slice 0 is theta = 0: band j holds row j
    o = np.concatenate([[0], np.cumsum(rl)])
    band = j0 - rmin[0]
    kept = z[o[band]:o[band + 1]].tolist()
    assert kept == [(2 * a + 1) << 15, (2 * b + 1) << 15]
    full = oref.RefCDDT(occ, n)
    _, rl_f, _ = full.export()
    assert rl_f[band] == b - a + 1                   # unpruned: every cell of the line


def test_pruned_update_rebuilds():
    rng = wl.rng_for(954, 0)
    occ = wl.random_map(rng, 40, 30, 0.2)
    n = 36
    pr = oref.RefCDDT(occ.copy(), n, prune=True)
    xs = rng.integers(0, 40, 60).astype(np.int32)
    ys = rng.integers(0, 30, 60).astype(np.int32)
    vs = rng.integers(0, 2, 60).astype(np.uint8)
    pr.update(xs, ys, vs)
    fresh = oref.RefCDDT(pr.occ.copy(), n, prune=True)
    for a, b in zip(pr.export(), fresh.export()):
        assert (a == b).all()


def test_pruning_shrinks_room_maps():
    """Memory drops markedly on room maps (the paper reports about 36-39% on its maps)."""
    occ = wl.building_map(wl.rng_for(955, 0), 300, 300)
    n = 108
    _, total, _ = oref.RefCDDT(occ, n, threads=4).sizes()
    _, pruned, _ = oref.RefCDDT(occ, n, threads=4, prune=True).sizes()
    assert pruned < 0.8 * total, (pruned, total)


def test_prune_and_zp16_not_combined():
    with pytest.raises(ValueError):
        oref.RefCDDT(np.zeros((4, 4), np.uint8), 8, zp16=True, prune=True)
