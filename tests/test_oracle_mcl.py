"""Pins for the oracle's motion model and systematic resampling (CPU only).

The paper names the motion and resampling steps of the particle filter
(Sec. I, Sec. VI) without formulas; the readings are in oracle/mcl_ref.c.
These tests tie them to facts that do not come from the oracle itself: the
library exp / sin / cos, closed forms of the motion model, the textbook
properties of systematic resampling and a brute-force pointer walk.
"""
import math

import numpy as np
import pytest

from oracle import ref as oref


# ---------------------------------------------------------------------------
# deterministic exp / sin / cos against the C library
# ---------------------------------------------------------------------------
def test_det_exp_matches_library_exp():
    xs = np.concatenate([-np.linspace(0, 64, 20001), -np.geomspace(1e-300, 64, 2000), [0.0, -0.5, -1e-17]])
    for x in xs:
        got, want = oref.det_exp_neg(float(x)), math.exp(float(x))
        # the reduction x log2(e) carries a rounding of relative size 2^-53, i.e. |x| 1.1e-16 absolute in the exponent
        assert abs(got - want) <= (4e-16 + 2e-16 * abs(float(x))) * want, (x, got, want)
    assert oref.det_exp_neg(0.0) == 1.0
    assert oref.det_exp_neg(-64.0001) == 0.0 and oref.det_exp_neg(float("-inf")) == 0.0
    assert oref.det_exp_neg(float("nan")) == 0.0


def test_det_sincos_matches_library():
    rng = np.random.default_rng(1)
    xs = np.concatenate([rng.uniform(-10, 10, 5000), rng.uniform(-1e3, 1e3, 2000),
                         np.arange(-16, 17) * (math.pi / 4), [0.0, -0.0, 1e-300]])
    for a in xs:
        s, c = oref.det_sincos(float(a))
        assert abs(s - math.sin(a)) <= 1e-15 * max(1.0, abs(a)) + 2e-16, (a, s, math.sin(a))
        assert abs(c - math.cos(a)) <= 1e-15 * max(1.0, abs(a)) + 2e-16, (a, c, math.cos(a))
    assert oref.det_sincos(0.0) == (0.0, 1.0)


# ---------------------------------------------------------------------------
# motion model
# ---------------------------------------------------------------------------
def _poses(n, seed=0):
    rng = np.random.default_rng(seed)
    return (rng.uniform(0, 500, n).astype(np.float32), rng.uniform(0, 500, n).astype(np.float32),
            rng.uniform(-math.pi, math.pi, n).astype(np.float32))


def test_motion_identity_and_pure_moves():
    px, py, pth = _poses(1000)
    z = np.zeros(1000, np.float32)
    x, y, t = oref.motion(px, py, pth, (0, 0, 0), z, z, z)
    assert (x == px).all() and (y == py).all() and (t == pth).all()     # exact: nothing to round
    # forward along +x at heading 0: exact
    h0 = np.zeros(1000, np.float32)
    x, y, t = oref.motion(px, py, h0, (2.5, 0, 0), z, z, z)
    assert (x == px + np.float32(2.5)).all() and (y == py).all()
    # heading wraps into [-pi, pi)
    x, y, t = oref.motion(px, py, pth, (0, 0, 7.0), z, z, z)
    assert (t >= -math.pi - 1e-6).all() and (t < math.pi + 1e-6).all()
    d = np.mod(t.astype(np.float64) - (pth.astype(np.float64) + 7.0) + math.pi, 2 * math.pi) - math.pi
    assert np.abs(d).max() < 1e-5


def test_motion_matches_textbook_formula():
    """Robot-frame odometry rotated by the heading, plus the noise (numpy float64 trig)."""
    n = 5000
    px, py, pth = _poses(n, 3)
    rng = np.random.default_rng(4)
    ex, ey, et = (rng.normal(0, s, n).astype(np.float32) for s in (0.05, 0.05, 0.02))
    dx, dy, dth = 0.7, -0.2, 0.05
    x, y, t = oref.motion(px, py, pth, (dx, dy, dth), ex, ey, et)
    th = pth.astype(np.float64)
    wx = px + np.cos(th) * np.float32(dx) - np.sin(th) * np.float32(dy) + ex
    wy = py + np.sin(th) * np.float32(dx) + np.cos(th) * np.float32(dy) + ey
    assert np.abs(x - wx).max() < 1e-4 and np.abs(y - wy).max() < 1e-4
    wt = np.mod(th + np.float32(dth) + et + math.pi, 2 * math.pi) - math.pi
    assert np.abs(np.mod(t - wt + math.pi, 2 * math.pi) - math.pi).max() < 1e-5


# ---------------------------------------------------------------------------
# systematic resampling
# ---------------------------------------------------------------------------
def _pointer_walk(q, total, u):
    """Textbook systematic resampling in integers: output j takes the first k with n C_(k+1) > s + j T."""
    n = len(q)
    s = ((u >> 12) * total) >> 20
    cum = np.cumsum([int(v) for v in q])
    out, k = [], 0
    for j in range(n):
        while n * int(cum[k]) <= s + j * total:
            k += 1
        out.append(k)
    return np.array(out, np.int32)


@pytest.mark.parametrize("seed", range(12))
def test_resample_equals_pointer_walk(seed):
    rng = np.random.default_rng(100 + seed)
    n = int(rng.choice([1, 2, 3, 7, 64, 65, 500, 2048]))
    logw = rng.normal(0, rng.uniform(0.1, 30), n).astype(np.float32) - np.float32(rng.uniform(0, 1000))
    if seed % 3 == 0 and n > 3:
        logw[rng.integers(0, n, n // 3)] = -np.inf
    u = int(rng.integers(0, 2**32))
    idx, x, y, t = oref.resample(logw, u, np.arange(n, dtype=np.float32), -np.arange(n, dtype=np.float32),
                                 np.full(n, 0.5, np.float32))
    q, total = oref.resample_weights(logw)
    assert (idx == _pointer_walk(q, total, u)).all()
    assert (x == idx.astype(np.float32)).all() and (y == -idx.astype(np.float32)).all() and (t == 0.5).all()


@pytest.mark.parametrize("seed", range(8))
def test_resample_copy_counts_are_floor_or_ceil(seed):
    """Each particle gets floor or ceil of n q_k / T copies, in source order, n in all."""
    rng = np.random.default_rng(200 + seed)
    n = int(rng.integers(1, 3000))
    logw = (rng.normal(0, 5, n) - 300).astype(np.float32)
    q, total = oref.resample_weights(logw)
    idx, *_ = oref.resample(logw, int(rng.integers(0, 2**32)), np.zeros(n), np.zeros(n), np.zeros(n))
    assert (np.diff(idx) >= 0).all() and idx.min() >= 0 and idx.max() < n
    counts = np.bincount(idx, minlength=n)
    assert counts.sum() == n
    lo = (n * q.astype(object)) // total
    hi = -((-n * q.astype(object)) // total)
    assert all(l <= c <= h for c, l, h in zip(counts, lo, hi))


def test_resample_special_cases():
    n = 1000
    z = np.zeros(n, np.float32)
    # equal weights: every particle exactly once, whatever u
    for u in (0, 1, 2**31, 2**32 - 1):
        idx, *_ = oref.resample(np.full(n, -3.5, np.float32), u, z, z, z)
        assert (idx == np.arange(n)).all()
    # one finite weight: every output copies it
    lw = np.full(n, -np.inf, np.float32)
    lw[417] = -10.0
    idx, *_ = oref.resample(lw, 12345, z, z, z)
    assert (idx == 417).all()
    # nothing finite: treated as equal weights
    idx, *_ = oref.resample(np.full(n, np.nan, np.float32), 999, z, z, z)
    assert (idx == np.arange(n)).all()
    # u = 0 closed form: a_k = ceil(n C_k / T)
    rng = np.random.default_rng(7)
    lw = rng.normal(0, 2, n).astype(np.float32)
    q, total = oref.resample_weights(lw)
    idx, *_ = oref.resample(lw, 0, z, z, z)
    cum = np.concatenate([[0], np.cumsum(q.astype(np.int64))])
    a = -((-n * cum) // total)
    want = np.repeat(np.arange(n), np.diff(a))
    assert (idx == want).all()
    # the largest weight quantizes to exactly 2^20
    assert q.max() == 1 << 20
    # quantization follows its definition with the library exp (ties aside)
    m = lw.max()
    ref_q = np.floor(np.exp(lw.astype(np.float64) - np.float64(m)) * 2.0**20).astype(np.uint64)
    assert (np.abs(q.astype(np.int64) - ref_q.astype(np.int64)) <= 1).all()
    with pytest.raises(ValueError):
        oref.resample(np.zeros((1 << 20) + 1, np.float32), 0, np.zeros(1), np.zeros(1), np.zeros(1))

