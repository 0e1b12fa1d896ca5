"""Seeded synthetic inputs for CDDT ray casting and the beam sensor model.

This module only draws inputs: occupancy grids shaped like the paper's maps (a
rectangle-cluttered "Synthetic"-style grid and a room/corridor "Basement"-style
floor), particle poses, the 270-degree lidar ray layout, a beam-model log table,
observed ranges and map-toggle operations.  It holds none of the CDDT arithmetic
(no projection, no zero points, no search): both the test oracle and the GPU
library consume what it produces, and neither is imported here.

Every generator takes a ``numpy.random.Generator``; ``rng_for(config, stream)``
builds one from ``SeedSequence([config, stream])`` so each workload and each
input stream of a workload is reproducible on its own.
"""
from __future__ import annotations

import math

import numpy as np

# Workload ids used as the first SeedSequence word.
SMALL, FLOOR, BATCHED, UPDATES, SERVING, SUITES = 1, 2, 3, 4, 5, 6

# Stream ids (second SeedSequence word).
S_MAP, S_POSES, S_TABLE, S_OBS, S_OPS, S_SPEC, S_ARRIVALS, S_MOTION = range(8)


def rng_for(config: int, stream: int, extra: int | None = None) -> np.random.Generator:
    words = [int(config), int(stream)] + ([] if extra is None else [int(extra)])
    return np.random.default_rng(np.random.SeedSequence(words))


# --------------------------------------------------------------------------
# Maps
# --------------------------------------------------------------------------
def rect_map(rng: np.random.Generator, width: int = 256, height: int = 256,
             n_rects: int = 40, side: tuple[int, int] = (4, 20)) -> np.ndarray:
    """Border wall plus filled axis-aligned rectangles (sides uniform in `side`)."""
    occ = np.zeros((height, width), np.uint8)
    occ[0, :] = occ[-1, :] = 1
    occ[:, 0] = occ[:, -1] = 1
    for _ in range(n_rects):
        w = int(rng.integers(side[0], side[1] + 1))
        h = int(rng.integers(side[0], side[1] + 1))
        x0 = int(rng.integers(0, max(1, width - w + 1)))
        y0 = int(rng.integers(0, max(1, height - h + 1)))
        occ[y0:y0 + h, x0:x0 + w] = 1
    return occ


def building_map(rng: np.random.Generator, width: int, height: int,
                 room: tuple[int, int] = (60, 120), corridor: tuple[int, int] = (3, 6),
                 door: tuple[int, int] = (3, 6), corridor_prob: float = 0.25) -> np.ndarray:
    """Room/corridor floor plan with one-cell-thick walls.

    A rectangle is split recursively along its longer side until it is no longer
    than a per-room limit drawn from `room`; a split leaves at least room[0]//2
    cells on each side, so finished rooms have sides of roughly 30 to 120 cells
    and the floor is about 4% occupied.  A split is a single wall or, with
    probability `corridor_prob`, two parallel walls `corridor` cells apart that
    enclose a corridor left unsplit.  Every wall gets one or two door gaps of
    `door` cells.  The map edge is a wall.
    """
    occ = np.zeros((height, width), np.uint8)
    occ[0, :] = occ[-1, :] = 1
    occ[:, 0] = occ[:, -1] = 1
    half = room[0] // 2

    def wall(vertical: bool, p: int, a0: int, a1: int) -> None:
        span = a1 - a0
        if vertical:
            occ[a0:a1, p] = 1
        else:
            occ[p, a0:a1] = 1
        n_doors = 1 if span < 2 * room[1] else 2
        for _ in range(n_doors):
            dw = int(rng.integers(door[0], door[1] + 1))
            if span <= dw + 2:
                continue
            g = int(rng.integers(a0 + 1, a1 - dw))
            if vertical:
                occ[g:g + dw, p] = 0
            else:
                occ[p, g:g + dw] = 0

    stack = [(1, 1, width - 1, height - 1)]  # interior cells [x0,x1) x [y0,y1)
    while stack:
        x0, y0, x1, y1 = stack.pop()
        w, h = x1 - x0, y1 - y0
        limit = int(rng.integers(room[0], room[1] + 1))
        if max(w, h) <= limit:
            continue
        vertical = w >= h
        length = w if vertical else h
        lo = x0 if vertical else y0
        c = int(rng.integers(corridor[0], corridor[1] + 1))
        use_corridor = rng.random() < corridor_prob and length > 2 * half + c + 2
        if use_corridor:
            p = int(rng.integers(lo + half, lo + length - half - c - 1))
            q = p + c + 1
            if vertical:
                wall(True, p, y0, y1)
                wall(True, q, y0, y1)
                stack.append((x0, y0, p, y1))
                stack.append((q + 1, y0, x1, y1))
            else:
                wall(False, p, x0, x1)
                wall(False, q, x0, x1)
                stack.append((x0, y0, x1, p))
                stack.append((x0, q + 1, x1, y1))
        else:
            p = int(rng.integers(lo + half, lo + length - half))
            if vertical:
                wall(True, p, y0, y1)
                stack.append((x0, y0, p, y1))
                stack.append((p + 1, y0, x1, y1))
            else:
                wall(False, p, x0, x1)
                stack.append((x0, y0, x1, p))
                stack.append((x0, p + 1, x1, y1))
    return occ


def random_map(rng: np.random.Generator, width: int, height: int, density: float) -> np.ndarray:
    """i.i.d. Bernoulli occupancy, used for small property tests."""
    return (rng.random((height, width)) < density).astype(np.uint8)


# --------------------------------------------------------------------------
# Poses, rays, sensor model, observations
# --------------------------------------------------------------------------
def free_poses(rng: np.random.Generator, occ: np.ndarray, n: int):
    """float32 poses: a uniform free cell plus a uniform offset inside it, theta in [0, 2pi)."""
    h, w = occ.shape
    free = np.flatnonzero(occ.ravel() == 0)
    if free.size == 0:
        raise ValueError("map has no free cell")
    idx = free[rng.integers(0, free.size, n)]
    ci = (idx % w).astype(np.float32)
    cj = (idx // w).astype(np.float32)
    u = rng.random(n, dtype=np.float32)
    v = rng.random(n, dtype=np.float32)
    x = np.minimum(ci + u, np.nextafter(ci + np.float32(1), np.float32(0)))
    y = np.minimum(cj + v, np.nextafter(cj + np.float32(1), np.float32(0)))
    th = (rng.random(n) * (2.0 * math.pi)).astype(np.float32)
    return x.astype(np.float32), y.astype(np.float32), th


def grid_states(width: int, height: int, theta_bins: int, stride: int = 1):
    """The "grid" suite's queries (Sec. VI): every stride-th cell centre in x and y, at every bin centre angle
    (float32 of 2 pi k / n computed in double); k slowest, then y, then x.  float32 (x, y, theta)."""
    xs = np.arange(0, width, stride, dtype=np.float64) + 0.5
    ys = np.arange(0, height, stride, dtype=np.float64) + 0.5
    th = (2.0 * math.pi * np.arange(theta_bins, dtype=np.float64) / theta_bins).astype(np.float32)
    k, j, i = np.meshgrid(np.arange(theta_bins), np.arange(ys.size), np.arange(xs.size), indexing="ij")
    return (xs[i.ravel()].astype(np.float32), ys[j.ravel()].astype(np.float32), th[k.ravel()])


def random_states(rng: np.random.Generator, width: int, height: int, count: int):
    """The "random" suite's queries (Sec. VI): states uniform over [0, W) x [0, H) x [0, 2 pi), float32 (occupied
    cells included: their casts return 0)."""
    x = (rng.random(count) * width).astype(np.float32)
    y = (rng.random(count) * height).astype(np.float32)
    x = np.minimum(x, np.nextafter(np.float32(width), np.float32(0)))
    y = np.minimum(y, np.nextafter(np.float32(height), np.float32(0)))
    th = (rng.random(count) * (2.0 * math.pi)).astype(np.float32)
    return x, y, th


def ray_offsets(n_rays: int = 61, fov: float = 1.5 * math.pi) -> np.ndarray:
    """Evenly spaced lidar bearings over `fov`, centred on the heading (double, then float32)."""
    if n_rays == 1:
        return np.zeros(1, np.float32)
    step = fov / (n_rays - 1)
    return np.array([-fov / 2.0 + r * step for r in range(n_rays)], np.float64).astype(np.float32)


def beam_params(rng: np.random.Generator) -> dict:
    """Mixture weights (hit, short, max, random) summing to 1 with a random floor of at least 0.02."""
    w_hit = rng.uniform(0.6, 0.8)
    w_short = rng.uniform(0.05, 0.15)
    w_max = rng.uniform(0.02, 0.08)
    w_rand = max(1.0 - w_hit - w_short - w_max, 0.02)
    tot = w_hit + w_short + w_max + w_rand
    return dict(w_hit=w_hit / tot, w_short=w_short / tot, w_max=w_max / tot, w_rand=w_rand / tot,
                sigma=rng.uniform(4.0, 10.0), lam=rng.uniform(0.005, 0.05))


def beam_table(max_range: int, params: dict) -> np.ndarray:
    """Discretised four-part beam model as a float32 log table laid out [obs][expected].

    Column e (expected range) is a distribution over the observation z in
    0..max_range: a Gaussian around e, an exponential short-reading term on
    z <= e, a spike at z = max_range and a uniform floor, mixed with the given
    weights and renormalised; entries are log-probabilities computed in double.
    """
    m = max_range
    z = np.arange(m + 1, dtype=np.float64)[:, None]
    e = np.arange(m + 1, dtype=np.float64)[None, :]
    hit = np.exp(-((z - e) ** 2) / (2.0 * params["sigma"] ** 2))
    hit /= hit.sum(axis=0, keepdims=True)
    short = np.where(z <= e, params["lam"] * np.exp(-params["lam"] * z), 0.0)
    short /= short.sum(axis=0, keepdims=True)
    pmax = (z == m).astype(np.float64) * np.ones_like(e)
    prand = np.full_like(hit, 1.0 / (m + 1))
    p = (params["w_hit"] * hit + params["w_short"] * short
         + params["w_max"] * pmax + params["w_rand"] * prand)
    p /= p.sum(axis=0, keepdims=True)
    return np.log(p).astype(np.float32)


def march_ranges(occ: np.ndarray, x: float, y: float, thetas: np.ndarray, max_range: int,
                 step: float = 0.05) -> np.ndarray:
    """Coarse fixed-step marching from one pose, used only to synthesise noisy observations."""
    h, w = occ.shape
    t = np.arange(0.0, max_range + step, step)
    px = x + np.cos(thetas.astype(np.float64))[:, None] * t[None, :]
    py = y + np.sin(thetas.astype(np.float64))[:, None] * t[None, :]
    ix = np.floor(px).astype(np.int64)
    iy = np.floor(py).astype(np.int64)
    inside = (ix >= 0) & (ix < w) & (iy >= 0) & (iy < h)
    hit = np.zeros_like(inside)
    hit[inside] = occ[iy[inside], ix[inside]] != 0
    hit |= ~inside
    first = np.where(hit.any(axis=1), hit.argmax(axis=1), t.size - 1)
    return np.minimum(np.rint(t[first]), max_range).astype(np.int64)


def observations(rng: np.random.Generator, occ: np.ndarray, offsets: np.ndarray, max_range: int,
                 noise_sigma: float = 8.0):
    """Observed ranges of one hidden free pose: marched range + N(0, sigma^2), rounded, clamped."""
    hx, hy, hth = free_poses(rng, occ, 1)
    thetas = (hth[0].astype(np.float64) + offsets.astype(np.float64))
    r = march_ranges(occ, float(hx[0]), float(hy[0]), thetas, max_range)
    z = np.rint(r + rng.normal(0.0, noise_sigma, r.size))
    return np.clip(z, 0, max_range).astype(np.int32), (float(hx[0]), float(hy[0]), float(hth[0]))


def toggle_ops(rng: np.random.Generator, occ: np.ndarray, k: int):
    """k uniformly random cells (repeats allowed) each set to 1 - current value."""
    h, w = occ.shape
    xs = rng.integers(0, w, k).astype(np.int32)
    ys = rng.integers(0, h, k).astype(np.int32)
    vals = (1 - (occ[ys, xs] != 0)).astype(np.uint8)
    return xs, ys, vals


def apply_ops(occ: np.ndarray, xs, ys, vals) -> None:
    """Apply ops in array order (later writes win) to a host grid in place."""
    for x, y, v in zip(xs.tolist(), ys.tolist(), vals.tolist()):
        occ[y, x] = 1 if v else 0


# --------------------------------------------------------------------------
# Whole-workload recipes
# --------------------------------------------------------------------------
THETA_CHOICES = (108, 200, 360)


def batched_specs(rng: np.random.Generator, n_filters: int = 64, side=(512, 4000),
                  particles=(500, 20000)):
    """Per-filter (map side, theta bins, particle count) for the many-filter workload."""
    specs = []
    for _ in range(n_filters):
        s = int(rng.integers(side[0], side[1] + 1))
        n = int(THETA_CHOICES[int(rng.integers(0, len(THETA_CHOICES)))])
        p = int(round(math.exp(rng.uniform(math.log(particles[0]), math.log(particles[1])))))
        specs.append(dict(side=s, theta_bins=n, particles=p))
    return specs


def map_stats(occ: np.ndarray) -> dict:
    return dict(width=int(occ.shape[1]), height=int(occ.shape[0]),
                occupancy=float((occ != 0).mean()))
