"""Oracle pins for the incremental update (Sec. IV-D) and the beam sensor model (Sec. VI).

Update: the incrementally maintained structure must equal a fresh build of the
new grid (rows as multisets), in both oracle implementations, over random op
sequences with repeated cells.  Sensor model: the synthetic beam table is a
proper distribution per expected range, and the per-particle log-weight is the
sum over rays of table[obs][expected] with the ray angle theta + offset.
"""
import math

import numpy as np
import pytest

from oracle import exact as ex
from paper_1705_01167_amd import workloads as wl


def _same(a, b):
    return all((x == y).all() for x, y in zip(a, b))


@pytest.mark.parametrize("seed", range(8))
@pytest.mark.parametrize("full_map", [False, True])
def test_update_equals_rebuild(seed, full_map, oracle_ref):
    rng = wl.rng_for(201, seed)
    w, h = int(rng.integers(3, 22)), int(rng.integers(3, 22))
    occ = wl.random_map(rng, w, h, float(rng.uniform(0.1, 0.6)))
    n = int(rng.choice([4, 8, 36, 108]))
    py = ex.PlainCDDT(occ, n, full_map=full_map)
    cc = oracle_ref.RefCDDT(occ, n, full_map=full_map)
    cur = occ.copy()
    for step in range(4):
        k = int(rng.integers(1, 25))
        xs = rng.integers(0, w, k).astype(np.int32)
        ys = rng.integers(0, h, k).astype(np.int32)
        if k > 2:                      # repeat a cell inside the batch: last write wins
            xs[-1], ys[-1] = xs[0], ys[0]
        vals = rng.integers(0, 2, k).astype(np.uint8)
        py.update(xs, ys, vals)
        cc.update(xs, ys, vals)
        wl.apply_ops(cur, xs, ys, vals)
        fresh = ex.PlainCDDT(cur, n, full_map=full_map)
        assert (py.occ == cur).all()
        assert _same(py.export(), fresh.export())
        assert _same(cc.export(), fresh.export())
        xq = rng.uniform(0, w, 300).astype(np.float32)
        yq = rng.uniform(0, h, 300).astype(np.float32)
        tq = rng.uniform(0, 7, 300).astype(np.float32)
        assert (cc.cast(xq, yq, tq, 40) == fresh.cast_many(xq, yq, tq, 40)).all()


def test_update_reveals_interior_cell(oracle_ref):
    """Removing an edge cell of a 3x3 block makes the hidden centre an edge (Sec. IV-D)."""
    occ = np.zeros((7, 7), np.uint8)
    occ[2:5, 2:5] = 1
    pc = ex.PlainCDDT(occ, 8)
    before = sum(len(r) for s in pc.rows for r in s)
    pc.update([2], [2], [0])
    after_occ = occ.copy()
    after_occ[2, 2] = 0
    fresh = ex.PlainCDDT(after_occ, 8)
    assert _same(pc.export(), fresh.export())
    # the centre (3, 3) is now an edge: theta = 0 band 3 holds it
    assert (2 * 3 + 1) << 15 in pc.rows[0][3 - pc.row_min[0]]
    assert sum(len(r) for s in pc.rows for r in s) != before
    # and re-occupying hides it again
    pc.update([2], [2], [1])
    assert _same(pc.export(), ex.PlainCDDT(occ, 8).export())


def test_update_rejects_off_map(oracle_ref):
    occ = np.zeros((4, 5), np.uint8)
    cc = oracle_ref.RefCDDT(occ, 4)
    with pytest.raises(ValueError):
        cc.update(np.array([1, 5], np.int32), np.array([0, 0], np.int32), np.array([1, 1], np.uint8))
    assert cc.sizes()[1] == 0   # nothing applied


def test_update_noop_and_same_value(oracle_ref):
    rng = wl.rng_for(202, 0)
    occ = wl.random_map(rng, 12, 9, 0.3)
    cc = oracle_ref.RefCDDT(occ, 36)
    ref = cc.export()
    ys, xs = np.nonzero(occ)
    assert cc.update(xs.astype(np.int32), ys.astype(np.int32), np.ones(xs.size, np.uint8)) == 0
    assert cc.update(np.zeros(0, np.int32), np.zeros(0, np.int32), np.zeros(0, np.uint8)) == 0
    assert _same(cc.export(), ref)
    # set then reset in one batch: last write wins -> no change
    x0, y0 = int(xs[0]), int(ys[0])
    cc.update(np.array([x0, x0], np.int32), np.array([y0, y0], np.int32), np.array([0, 1], np.uint8))
    assert _same(cc.export(), ref)


# ---------------------------------------------------------------------------
# Sensor model
# ---------------------------------------------------------------------------
def test_beam_params_are_a_mixture():
    """Every draw is a proper mixture (the random floor never goes negative)."""
    for seed in range(500):
        p = wl.beam_params(wl.rng_for(204, seed))
        w = [p["w_hit"], p["w_short"], p["w_max"], p["w_rand"]]
        assert min(w) > 0 and abs(sum(w) - 1.0) < 1e-12 and p["w_rand"] >= 0.019


@pytest.mark.parametrize("seed", range(3))
def test_beam_table_is_a_distribution(seed):
    p = wl.beam_params(wl.rng_for(203, seed))
    assert p["w_rand"] > 0 and 4 <= p["sigma"] <= 10 and 0.005 <= p["lam"] <= 0.05
    for m in (0, 1, 30, 500):
        t = wl.beam_table(m, p)
        assert t.shape == (m + 1, m + 1) and t.dtype == np.float32
        assert np.isfinite(t).all() and (t <= 0).all()
        col = np.exp(t.astype(np.float64)).sum(axis=0)   # sum over observations per expected range
        assert np.allclose(col, 1.0, atol=1e-5 * (m + 1))
        if m >= 30:
            e = m // 2   # the Gaussian term makes z = e the most likely non-max observation
            assert t[e, e] == t[:m, e].max()
            assert t[m, e] > t[m - 1, e]   # max-range spike


def test_particle_log_weight(oracle_ref):
    rng = wl.rng_for(204, 0)
    occ = wl.rect_map(rng, 40, 30, n_rects=6, side=(2, 6))
    n, M = 36, 60
    off = wl.ray_offsets(61)
    obs = rng.integers(0, M + 1, 61).astype(np.int32)
    obs[3] = -5          # clamped to 0
    obs[4] = M + 9       # clamped to M
    # an asymmetric table pins the [observation][expected] orientation
    z = np.arange(M + 1)[:, None]
    e = np.arange(M + 1)[None, :]
    table = (-(z * 1000 + e) * 1e-3).astype(np.float32)
    px, py_, pth = wl.free_poses(rng, occ, 25)
    bf = ex.BruteForce(occ, n)
    cc = oracle_ref.RefCDDT(occ, n)
    logw, ranges = cc.weight(px, py_, pth, off, obs, table, M, want_ranges=True)
    for p in range(25):
        want = 0.0
        for r in range(61):
            th = np.float32(pth[p] + off[r])
            d = bf.cast(px[p], py_[p], th, M)
            assert ranges[p, r] == d
            zz = min(max(int(obs[r]), 0), M)
            want += float(np.float32(-(zz * 1000 + d) * 1e-3))
        assert abs(logw[p] - want) < 1e-9
        got_py, _ = ex.particle_log_weight(bf, px[p], py_[p], pth[p], off, obs, table.ravel(), M)
        assert abs(got_py - want) < 1e-9


def test_weight_threads_agree(oracle_ref):
    rng = wl.rng_for(205, 0)
    occ = wl.rect_map(rng, 64, 64, n_rects=10)
    cc = oracle_ref.RefCDDT(occ, 108)
    off = wl.ray_offsets(61)
    obs = rng.integers(0, 101, 61).astype(np.int32)
    table = wl.beam_table(100, wl.beam_params(rng))
    px, py_, pth = wl.free_poses(rng, occ, 500)
    a = cc.weight(px, py_, pth, off, obs, table, 100, threads=1)
    b = cc.weight(px, py_, pth, off, obs, table, 100, threads=4)
    assert (a == b).all()
    c = cc.cast(px, py_, pth, 100, threads=1)
    d = cc.cast(px, py_, pth, 100, threads=3)
    assert (c == d).all()
