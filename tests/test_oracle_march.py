"""The oracle of the cell-walk comparator (a comparison system of Sec. II):
pinned by closed forms on axis-aligned and diagonal rays, and by dense
sampling along the ray on random maps (independent of the traversal)."""
import math

import numpy as np

from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl


def test_axis_rays_closed_form():
    occ = np.zeros((10, 12), np.uint8)
    occ[1, 7] = 1          # in row 1, to the right of x = 2.3: entry at x = 7, t = 4.7 -> 5
    occ[6, 3] = 1          # in column 3, above y = 0.25: entry at y = 6, t = 5.75 -> 6
    assert oref.march_cast(occ, 2.3, 1.5, 0.0, 100) == 5
    assert oref.march_cast(occ, 3.5, 0.25, np.float32(math.pi / 2), 100) == 6
    assert oref.march_cast(occ, 9.6, 1.5, np.float32(math.pi), 100) == 2    # from the right: 9.6 - 8 = 1.6 -> 2
    assert oref.march_cast(occ, 2.3, 1.5, 0.0, 3) == 3                       # capped
    assert oref.march_cast(occ, 2.3, 2.5, 0.0, 100) == 100                   # leaves the map
    assert oref.march_cast(occ, 7.5, 1.5, 0.0, 100) == 0                     # starts in an obstacle
    assert oref.march_cast(occ, -0.1, 1.5, 0.0, 100) == 0                    # off the map
    assert oref.march_cast(occ, 2.3, 1.5, float("nan"), 100) == 0
    assert oref.march_cast(occ, 2.3, 1.5, 2e6, 100) == 0


def test_diagonal_closed_form():
    # the ray from (0.5, 1.25) at 45 degrees is y = x + 0.75 (to rounding): it passes cell (5, 4) (x in [5, 6),
    # y in [4, 5)) above it, since at x = 5 it is already at y = 5.75, and leaves the 8 x 8 map through y = 8
    occ = np.zeros((8, 8), np.uint8)
    occ[4, 5] = 1
    assert oref.march_cast(occ, 0.5, 1.25, np.float32(math.pi / 4), 50) == 50
    # cell (4, 5) (x in [4, 5), y in [5, 6)) is entered through its bottom edge y = 5 at x = 4.25
    occ[5, 4] = 1
    t = (4.25 - 0.5) * math.sqrt(2.0)
    assert oref.march_cast(occ, 0.5, 1.25, np.float32(math.pi / 4), 50) == int(math.floor(t + 0.5)) == 5


def _sampled(occ, x, y, th, M, step=1e-4):
    """Entry distance by dense sampling along the ray (independent of the cell traversal)."""
    h, w = occ.shape
    s, c = oref.det_sincos(float(np.float32(th)))
    px, py = float(np.float32(x)), float(np.float32(y))
    if occ[int(math.floor(py)), int(math.floor(px))]:
        return 0.0
    t = 0.0
    while t < M + 1:
        t += step
        qx, qy = px + t * c, py + t * s
        if not (0 <= qx < w and 0 <= qy < h):
            return None
        if occ[int(math.floor(qy)), int(math.floor(qx))]:
            return t
    return None


def test_random_rays_match_sampling():
    rng = wl.rng_for(wl.SUITES, 99)
    occ = wl.random_map(rng, 24, 18, 0.12)
    M = 40
    x, y, th = wl.random_states(rng, 24, 18, 500)
    checked = 0
    for q in range(x.size):
        r = oref.march_cast(occ, x[q], y[q], th[q], M)
        t = _sampled(occ, x[q], y[q], th[q], M)
        if t is None:
            assert r == M
            continue
        if t == 0.0:
            assert r == 0
            continue
        if abs((t + 0.5) - round(t + 0.5)) < 1e-3:  # too close to a rounding boundary for the sampling step
            continue
        assert r == min(M, int(math.floor(t + 0.5))), (q, r, t)
        checked += 1
    assert checked > 150
