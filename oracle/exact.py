"""Exact CPU oracle for CDDT ray casting (test infrastructure only).

Only the tests, the smoke check and the benchmark's CPU-baseline leg use this
package; the GPU library never imports, links or calls it.

What is computed (Walsh & Karaman, "CDDT: Fast Approximate 2D Ray Casting for
Accelerated Localization"):

* Sec. III: a ray cast returns the distance from the query to the nearest
  occupied cell along the ray direction.  Sec. IV: the directional distance
  transform (DDT) rotates the scene by -theta so every cast runs along +x; each
  DDT row is a sawtooth whose zero points are obstacles, and the CDDT keeps only
  those zero points per row ("CDDT bin").  Sec. IV-A builds it by projecting
  every edge-map cell into each slice; Sec. IV-B answers a query with a
  successor search in the query's row; Sec. IV-C adds the theta / theta+pi
  symmetry (predecessor search), the edge-map reduction with the overlap check,
  and Sec. IV-D the incremental update with revealed-neighbour handling.

Integer reading used throughout (the paper leaves the numerics open; every
choice is listed in the design notes):

* cells (i, j) cover [i, i+1) x [j, j+1), grid row-major ``occ[j][i]``;
  theta runs from +x toward +y; n bins cover the full circle and the n/2
  slices 0 <= s < n/2 are stored (Sec. IV-C);
* per slice: C = llround(cos(2 pi s/n) 2^30), S = llround(sin(2 pi s/n) 2^30);
* zero point of cell (i, j): Z = ((2i+1) C + (2j+1) S) >> 15, the along-ray
  coordinate of the cell centre in units of 2^-16 cell;
* rows ("bins") a cell lands in: the rotated unit square's lateral extent
  [Yc - Hs, Yc + Hs) with Yc = (2j+1) C - (2i+1) S and Hs = |C| + |S| (units
  2^-31), intersected with half-open unit bands;
* a query (x, y, theta) in float32: xf = floor(x 2^16), yf = floor(y 2^16),
  bin k = floor(fl(fl(theta K) + 0.5)) mod n with K = float(n / 2 pi) and no
  fused multiply-add, slice s = k mod n/2, direction +1 if k < n/2 else -1,
  Xq = (xf C + yf S) >> 30, row r = (yf C - xf S) >> 46;
* successor (direction +1): smallest Z > Xq; predecessor (direction -1):
  largest Z < Xq; range = min(M, (|Z - Xq| + 2^15) >> 16), or M when no such Z;
* a query that is off the map, non-finite, |theta| >= 1e6, or inside an
  occupied cell (overlap check on the full grid) returns 0.

This module is the plain Python statement of those rules: a brute force over
every edge cell (the definition the CDDT accelerates) and a direct, unoptimised
CDDT (lists per row, ``sorted``, ``bisect``) following Sec. IV's algorithms.
"""
from __future__ import annotations

import bisect
import math
from dataclasses import dataclass, field

import numpy as np

ONE16 = 1 << 16
HALF16 = 1 << 15
TRIG_ONE = 1 << 30
THETA_LIMIT = np.float32(1e6)


# ---------------------------------------------------------------------------
# Tables
# ---------------------------------------------------------------------------
def llround(v: float) -> int:
    """Round half away from zero (C's llround)."""
    r = int(math.floor(abs(v) + 0.5))
    return r if v >= 0 else -r


def trig_table(n: int):
    """Fixed-point direction of each stored slice s in [0, n/2): angle 2 pi s / n."""
    cs, ss = [], []
    for s in range(n // 2):
        a = 2.0 * math.pi * s / n
        cs.append(llround(math.cos(a) * TRIG_ONE))
        ss.append(llround(math.sin(a) * TRIG_ONE))
    return cs, ss


def bin_scale(n: int) -> np.float32:
    """K = n / (2 pi) rounded once to float32."""
    return np.float32(n / (2.0 * math.pi))


def row_range(c: int, s: int, width: int, height: int):
    """Lowest and highest band index any point of the map rectangle can fall in."""
    lat = [(y * c - x * s) >> 30 for x in (0, width) for y in (0, height)]
    return min(lat), max(lat)


# ---------------------------------------------------------------------------
# Edge map (Sec. IV-C, erosion reduction)
# ---------------------------------------------------------------------------
def edge_map(occ: np.ndarray) -> np.ndarray:
    """Occupied cells that are not surrounded on all 8 sides by occupied in-map cells."""
    o = occ != 0
    h, w = o.shape
    pad = np.zeros((h + 2, w + 2), bool)
    pad[1:-1, 1:-1] = o
    interior = np.ones_like(o)
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            interior &= pad[1 + dj:1 + dj + h, 1 + di:1 + di + w]
    return o & ~interior


def is_edge(occ: np.ndarray, i: int, j: int) -> bool:
    h, w = occ.shape
    if occ[j, i] == 0:
        return False
    for dj in (-1, 0, 1):
        for di in (-1, 0, 1):
            if di == 0 and dj == 0:
                continue
            a, b = i + di, j + dj
            if a < 0 or b < 0 or a >= w or b >= h or occ[b, a] == 0:
                return True
    return False


# ---------------------------------------------------------------------------
# Projection of one cell (Sec. IV-A)
# ---------------------------------------------------------------------------
def cell_zero_point(i: int, j: int, c: int, s: int) -> int:
    return ((2 * i + 1) * c + (2 * j + 1) * s) >> 15


def cell_rows(i: int, j: int, c: int, s: int):
    """Inclusive band range covered by the rotated cell square."""
    yc = (2 * j + 1) * c - (2 * i + 1) * s
    hs = abs(c) + abs(s)
    return (yc - hs) >> 31, (yc + hs - 1) >> 31


# ---------------------------------------------------------------------------
# Query pre-processing (Sec. IV-B)
# ---------------------------------------------------------------------------
@dataclass
class Query:
    valid: bool          # False -> answer 0 (off map, non-finite, absurd theta, inside obstacle)
    k: int = 0           # theta bin over the full circle
    s: int = 0           # stored slice
    sigma: int = 1       # +1 successor, -1 predecessor
    xf: int = 0
    yf: int = 0
    xq: int = 0          # along-ray coordinate, units 2^-16
    r: int = 0           # band index


def theta_bin(theta: np.float32, n: int) -> int:
    t = np.float32(theta) * bin_scale(n)          # float32 product, round to nearest
    u = np.float32(t) + np.float32(0.5)           # separate float32 add (no FMA)
    return int(math.floor(float(u))) % n          # Python % is the Euclidean remainder here


def prepare(occ: np.ndarray, n: int, tabs, x, y, theta) -> Query:
    h, w = occ.shape
    x = np.float32(x)
    y = np.float32(y)
    theta = np.float32(theta)
    if not (abs(theta) < THETA_LIMIT):
        return Query(False)
    if not (x >= 0 and x < np.float32(w) and y >= 0 and y < np.float32(h)):
        return Query(False)
    xf = int(math.floor(float(x * np.float32(65536.0))))
    yf = int(math.floor(float(y * np.float32(65536.0))))
    if occ[yf >> 16, xf >> 16] != 0:
        return Query(False)
    k = theta_bin(theta, n)
    s = k % (n // 2)
    sigma = 1 if k < n // 2 else -1
    c, sn = tabs[0][s], tabs[1][s]
    xq = (xf * c + yf * sn) >> 30
    r = (yf * c - xf * sn) >> 46
    return Query(True, k, s, sigma, xf, yf, xq, r)


def finish(d: int | None, max_range: int) -> int:
    if d is None:
        return max_range
    return min(max_range, (d + HALF16) >> 16)


# ---------------------------------------------------------------------------
# Level-1 definition: brute force over the edge cells
# ---------------------------------------------------------------------------
class BruteForce:
    """Answers each query by scanning every edge cell; no per-row structure at all."""

    def __init__(self, occ: np.ndarray, n: int, full_map: bool = False):
        assert n % 2 == 0 and n >= 2
        self.occ = np.ascontiguousarray(occ)
        self.n = n
        self.tabs = trig_table(n)
        e = (self.occ != 0) if full_map else edge_map(self.occ)
        jj, ii = np.nonzero(e)
        self.ci = ii.astype(np.int64)
        self.cj = jj.astype(np.int64)

    def candidates(self, q: Query):
        c, s = self.tabs[0][q.s], self.tabs[1][q.s]
        two_i = 2 * self.ci + 1
        two_j = 2 * self.cj + 1
        z = (two_i * c + two_j * s) >> 15
        yc = two_j * c - two_i * s
        hs = abs(c) + abs(s)
        lo = (yc - hs) >> 31
        hi = (yc + hs - 1) >> 31
        inband = (lo <= q.r) & (q.r <= hi)
        return z[inband]

    def witness(self, q: Query):
        """Edge cells whose zero point decides the answer (for hit-witness checks)."""
        c, s = self.tabs[0][q.s], self.tabs[1][q.s]
        two_i = 2 * self.ci + 1
        two_j = 2 * self.cj + 1
        z = (two_i * c + two_j * s) >> 15
        yc = two_j * c - two_i * s
        hs = abs(c) + abs(s)
        inband = (((yc - hs) >> 31) <= q.r) & (q.r <= ((yc + hs - 1) >> 31))
        return self.ci[inband], self.cj[inband], z[inband]

    def cast(self, x, y, theta, max_range: int) -> int:
        q = prepare(self.occ, self.n, self.tabs, x, y, theta)
        if not q.valid:
            return 0
        z = self.candidates(q)
        if q.sigma > 0:
            ahead = z[z > q.xq]
            d = None if ahead.size == 0 else int(ahead.min()) - q.xq
        else:
            behind = z[z < q.xq]
            d = None if behind.size == 0 else q.xq - int(behind.max())
        return finish(d, max_range)

    def cast_many(self, xs, ys, ths, max_range: int) -> np.ndarray:
        return np.array([self.cast(a, b, t, max_range) for a, b, t in zip(xs, ys, ths)], np.int64)


# ---------------------------------------------------------------------------
# Plain CDDT following Sec. IV-A / IV-B / IV-C / IV-D
# ---------------------------------------------------------------------------
@dataclass
class PlainCDDT:
    occ: np.ndarray
    n: int
    full_map: bool = False
    prune: bool = False                # PCDDT: keep only zero points that some discrete state's cast returns
    tabs: tuple = field(init=False)
    row_min: list = field(init=False)
    nrows: list = field(init=False)
    rows: list = field(init=False)     # rows[s][r - row_min[s]] -> sorted list of int

    def __post_init__(self):
        assert self.n % 2 == 0 and self.n >= 2
        self.occ = np.array(self.occ, dtype=np.uint8, copy=True)
        self.tabs = trig_table(self.n)
        h, w = self.occ.shape
        self.row_min, self.nrows = [], []
        for s in range(self.n // 2):
            lo, hi = row_range(self.tabs[0][s], self.tabs[1][s], w, h)
            self.row_min.append(lo)
            self.nrows.append(hi - lo + 1)
        self._build()

    def _build(self) -> None:
        self.rows = [[[] for _ in range(self.nrows[s])] for s in range(self.n // 2)]
        cells = (self.occ != 0) if self.full_map else edge_map(self.occ)
        jj, ii = np.nonzero(cells)
        for s in range(self.n // 2):                       # for each stored theta
            for i, j in zip(ii.tolist(), jj.tolist()):     # for each edge-map cell
                self._touch(s, i, j, +1)
            for row in self.rows[s]:                       # initialise each bin
                row.sort()
        if self.prune:
            self._prune()

    def _search(self, q: Query):
        """The zero point a valid query's cast returns (successor or predecessor), or None."""
        row = self.rows[q.s][q.r - self.row_min[q.s]]
        if q.sigma > 0:
            k = bisect.bisect_right(row, q.xq)           # first zero point > Xq
            return None if k == len(row) else row[k]
        k = bisect.bisect_left(row, q.xq) - 1            # last zero point < Xq
        return None if k < 0 else row[k]

    def _prune(self) -> None:
        """PCDDT (Sec. IV-C): cast from every discrete state and keep, per band, only the
        zero points some cast returns.  States: the centre of every free cell under every
        theta bin, at the bin's centre angle 2 pi k / n."""
        used = [[set() for _ in range(self.nrows[s])] for s in range(self.n // 2)]
        free = np.argwhere(self.occ == 0)
        for k in range(self.n):
            theta = np.float32(2.0 * math.pi * k / self.n)
            for j, i in free.tolist():
                q = prepare(self.occ, self.n, self.tabs, np.float32(i + 0.5), np.float32(j + 0.5), theta)
                assert q.valid and q.k == k, "a state fell outside its bin"
                z = self._search(q)
                if z is not None:
                    used[q.s][q.r - self.row_min[q.s]].add(z)
        self.rows = [[sorted(u) for u in per_slice] for per_slice in used]

    def _touch(self, s: int, i: int, j: int, sign: int) -> None:
        c, sn = self.tabs[0][s], self.tabs[1][s]
        z = cell_zero_point(i, j, c, sn)
        lo, hi = cell_rows(i, j, c, sn)
        for r in range(lo, hi + 1):
            row = self.rows[s][r - self.row_min[s]]
            if sign > 0:
                bisect.insort(row, z)
            else:
                k = bisect.bisect_left(row, z)
                assert k < len(row) and row[k] == z, "removing a zero point that is absent"
                del row[k]

    def cast(self, x, y, theta, max_range: int) -> int:
        q = prepare(self.occ, self.n, self.tabs, x, y, theta)
        if not q.valid:
            return 0
        z = self._search(q)
        return finish(None if z is None else q.sigma * (z - q.xq), max_range)

    def cast_many(self, xs, ys, ths, max_range: int) -> np.ndarray:
        return np.array([self.cast(a, b, t, max_range) for a, b, t in zip(xs, ys, ths)], np.int64)

    def update(self, xs, ys, vals) -> None:
        """Sec. IV-D with the edge-map rule extended to both directions.

        Ops are applied in order (last write per cell wins).  Only cells within
        one step (8-neighbourhood) of a changed cell can change edge status; each
        such cell whose status flipped has its zero points removed from or
        inserted into every slice and every band it covers.  A pruned (PCDDT)
        structure is rebuilt and pruned again from the new grid.
        """
        h, w = self.occ.shape
        new = self.occ.copy()
        for x, y, v in zip(list(xs), list(ys), list(vals)):
            new[int(y), int(x)] = 1 if v else 0
        if self.prune:
            self.occ = new
            self._build()
            return
        changed = np.argwhere(new != self.occ)
        cand = set()
        for j, i in changed.tolist():
            for dj in (-1, 0, 1):
                for di in (-1, 0, 1):
                    a, b = i + di, j + dj
                    if 0 <= a < w and 0 <= b < h:
                        cand.add((a, b))
        status = {}
        for (a, b) in cand:
            if self.full_map:
                status[(a, b)] = (self.occ[b, a] != 0, new[b, a] != 0)
            else:
                status[(a, b)] = (is_edge(self.occ, a, b), is_edge(new, a, b))
        self.occ = new
        for (a, b), (old_e, new_e) in sorted(status.items()):
            if old_e and not new_e:
                for s in range(self.n // 2):
                    self._touch(s, a, b, -1)
        for (a, b), (old_e, new_e) in sorted(status.items()):
            if new_e and not old_e:
                for s in range(self.n // 2):
                    self._touch(s, a, b, +1)

    def export(self):
        """Canonical CSR: rows of all slices in (slice, band) order, each ascending."""
        lens, zeros = [], []
        for s in range(self.n // 2):
            for row in self.rows[s]:
                lens.append(len(row))
                zeros.extend(row)
        return (np.array(self.nrows, np.int64), np.array(lens, np.int64),
                np.array(zeros, np.int64))


# ---------------------------------------------------------------------------
# Sensor model: log-weight of one particle (beam model, Sec. VI)
# ---------------------------------------------------------------------------
def particle_log_weight(caster, x, y, theta, offsets, obs, log_table, max_range: int):
    """Sum over rays of log p(z_r | expected range), ray angle = fl(theta + offset)."""
    m1 = max_range + 1
    total = 0.0
    ranges = []
    for r in range(len(offsets)):
        th = np.float32(np.float32(theta) + np.float32(offsets[r]))
        d = caster.cast(x, y, th, max_range)
        z = min(max(int(obs[r]), 0), max_range)
        total += float(log_table[z * m1 + d])
        ranges.append(d)
    return total, ranges


# ---------------------------------------------------------------------------
# Independent textbook casts (pins, not CDDT)
# ---------------------------------------------------------------------------
def axis_scan(occ: np.ndarray, i: int, j: int, xq16: int, yq16: int, quarter: int, max_range: int):
    """Cardinal-direction cast by stepping cell to cell (quarter 0..3 = +x, +y, -x, -y).

    Distance is measured from the quantised query coordinate (units 2^-16) to
    the centre of the first occupied cell, rounded half up, capped at max_range.
    """
    h, w = occ.shape
    if occ[j, i]:
        return 0
    step = [(1, 0), (0, 1), (-1, 0), (0, -1)][quarter]
    a, b = i, j
    while True:
        a += step[0]
        b += step[1]
        if not (0 <= a < w and 0 <= b < h):
            return max_range
        if occ[b, a]:
            break
    if quarter == 0:
        d = (2 * a + 1) * HALF16 - xq16
    elif quarter == 1:
        d = (2 * b + 1) * HALF16 - yq16
    elif quarter == 2:
        d = xq16 - (2 * a + 1) * HALF16
    else:
        d = yq16 - (2 * b + 1) * HALF16
    return min(max_range, (d + HALF16) >> 16)


def grid_traversal(occ: np.ndarray, px: float, py: float, dx: float, dy: float):
    """Amanatides & Woo (1987) voxel walk in double.

    Returns (t_entry, i, j) of the first occupied cell the ray p + t d (t > 0)
    enters, or None if it leaves the map first.  The start cell is assumed free.
    """
    h, w = occ.shape
    i, j = int(math.floor(px)), int(math.floor(py))
    step_i = 1 if dx > 0 else -1
    step_j = 1 if dy > 0 else -1
    inf = float("inf")
    if dx != 0:
        nx = i + 1 if dx > 0 else i
        t_max_x = (nx - px) / dx
        t_dx = abs(1.0 / dx)
    else:
        t_max_x, t_dx = inf, inf
    if dy != 0:
        ny = j + 1 if dy > 0 else j
        t_max_y = (ny - py) / dy
        t_dy = abs(1.0 / dy)
    else:
        t_max_y, t_dy = inf, inf
    while True:
        if t_max_x < t_max_y:
            t = t_max_x
            i += step_i
            t_max_x += t_dx
        else:
            t = t_max_y
            j += step_j
            t_max_y += t_dy
        if not (0 <= i < w and 0 <= j < h):
            return None
        if occ[j, i]:
            return t, i, j


def dense_lut(occ: np.ndarray, n: int, max_range: int, caster) -> np.ndarray:
    """3D table of casts from every cell centre at every bin centre angle (uint16)."""
    h, w = occ.shape
    lut = np.zeros((n, h, w), np.uint16)
    for k in range(n):
        th = np.float32(2.0 * math.pi * k / n)
        for j in range(h):
            for i in range(w):
                lut[k, j, i] = caster.cast(np.float32(i + 0.5), np.float32(j + 0.5), th, max_range)
    return lut
