"""Bucket index (CDDT_FLAG_BUCKETS): the same ranges and weights as the oracle.

The bucket index only changes how a band is searched, so every result must be
bit-identical to the oracle's (and to the same map without the index), for
every bucket width, including widths where many buckets overflow and their
searches fall back to the band's search lines, and after map updates.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

RTOL = 1e-5


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    _torch()
    import torch
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _map(occ, n, **kw):
    from paper_1705_01167_amd import cddt
    return cddt.Map(_dev(occ), n, **kw)


def _queries(rng, w, h, k):
    x = rng.uniform(-2, w + 2, k).astype(np.float32)
    y = rng.uniform(-2, h + 2, k).astype(np.float32)
    th = rng.uniform(-40, 40, k).astype(np.float32)
    x[:4] = [np.nan, -0.0, np.float32(w), np.float32(w) - np.float32(1e-3)]
    x[4:100] = np.floor(x[4:100])                       # cell edges
    th[4:100] = (2 * math.pi * rng.integers(0, 4, 96) / 4).astype(np.float32)
    return x, y, th


@pytest.mark.parametrize("seed", range(8))
def test_bucket_tiny_maps(seed):
    """Random small maps and bucket widths 2^4..2^10 (wide buckets overflow): casts exact."""
    rng = wl.rng_for(701, seed)
    w, h = int(rng.integers(1, 90)), int(rng.integers(1, 90))
    occ = wl.random_map(rng, w, h, float(rng.uniform(0.0, 0.6)))
    n = int(rng.choice([2, 4, 8, 36, 108, 200, 360]))
    lb = int(rng.integers(4, 11))
    full = bool(rng.integers(0, 2))
    M = int(rng.choice([0, 7, 100, 65535]))
    _say(f"bucket tiny seed={seed} {w}x{h} n={n} log2={lb} full={full} M={M}")
    rm = oref.RefCDDT(occ, n, full_map=full)
    gb = _map(occ, n, full_map=full, buckets=lb)
    info = gb.info()
    assert info["bucket_log2"] == lb and info["bucket_lines"] > 0 and info["bucket_lines"] % info["rows"] == 0
    x, y, th = _queries(rng, w, h, 20000 + int(rng.integers(0, 77)))
    want = rm.cast(x, y, th, M, threads=4)
    got = gb.cast(_dev(x), _dev(y), _dev(th), M).cpu().numpy()
    assert (got == want).all(), f"{(got != want).sum()} rays differ"


@pytest.mark.parametrize("lb", [0, 5, 10])
def test_bucket_floor_2000(lb):
    """2000^2 floor, 200 bins, 2500 particles x 61 rays: ranges exact, weights within 1e-5."""
    occ = wl.building_map(wl.rng_for(wl.FLOOR, wl.S_MAP), 2000, 2000)
    n, M = 200, 500
    _say(f"bucket floor 2000 log2={lb}: builds")
    rm = oref.RefCDDT(occ, n, threads=8)
    gb = _map(occ, n, buckets=lb)
    info = gb.info()
    _say(f"bucket floor 2000: {info['bucket_lines']} lines, {info['bucket_overflow']} overflow")
    if lb == 10:
        assert info["bucket_overflow"] > 0          # the fallback path is exercised
    off = wl.ray_offsets(61)
    px, py, pth = wl.free_poses(wl.rng_for(wl.FLOOR, wl.S_POSES), occ, 2500)
    table = wl.beam_table(M, wl.beam_params(wl.rng_for(wl.FLOOR, wl.S_TABLE)))
    obs, _ = wl.observations(wl.rng_for(wl.FLOOR, wl.S_OBS), occ, off, M)
    ref_lw, ref_r = rm.weight(px, py, pth, off, obs, table, M, threads=8, want_ranges=True)
    lw, rr = gb.weight(_dev(px), _dev(py), _dev(pth), _dev(off), _dev(obs), _dev(table), M, ranges=True)
    rr = rr.cpu().numpy()
    assert (rr == ref_r).all(), f"{(rr != ref_r).sum()} ranges differ"
    lw = lw.cpu().numpy().astype(np.float64)
    assert (np.abs(lw - ref_lw) <= RTOL * np.maximum(1.0, np.abs(ref_lw))).all()


def test_bucket_overflow_count_matches_definition():
    """bucket_overflow equals the number of buckets holding more than 30 keys, counted from the oracle."""
    occ = wl.building_map(wl.rng_for(702, 0), 600, 500)
    n, lb = 108, 8
    rm = oref.RefCDDT(occ, n)
    gb = _map(occ, n, buckets=lb)
    c, s, rmin, nrows, _ = rm.tables()
    _, rl, zz = rm.export()
    offs = np.concatenate([[0], np.cumsum(rl)])
    h, w = occ.shape
    nb = 1
    zlo_all = []
    for k in range(n // 2):
        C, S = int(c[k]), int(s[k])
        wc, hs = (w << 16) * C, (h << 16) * S
        zlo, zhi = (min(0, wc) + min(0, hs)) >> 30, (max(0, wc) + max(0, hs)) >> 30
        zlo_all.append(zlo)
        nb = max(nb, ((zhi - zlo) >> (16 + lb)) + 1)
    over, row = 0, 0
    for k in range(n // 2):
        for _ in range(int(nrows[k])):
            keys = zz[offs[row]:offs[row + 1]].astype(np.int64)
            row += 1
            if keys.size:
                over += int((np.bincount((keys - zlo_all[k]) >> (16 + lb), minlength=nb) > 30).sum())
    info = gb.info()
    assert info["bucket_lines"] == info["rows"] * nb
    assert info["bucket_overflow"] == over


@pytest.mark.parametrize("seed", range(4))
def test_bucket_updates_match_oracle(seed):
    """Random toggles on a bucket map (default and a narrow width): casts equal the oracle after every step."""
    rng = wl.rng_for(703, seed)
    w, h = int(rng.integers(40, 160)), int(rng.integers(40, 160))
    occ = wl.random_map(rng, w, h, 0.15)
    n = int(rng.choice([36, 108, 200]))
    lb = int(rng.choice([0, 4]))
    static = bool(rng.integers(0, 2))
    M = 300
    _say(f"bucket updates seed={seed} {w}x{h} n={n} log2={lb} static={static}")
    rm = oref.RefCDDT(occ.copy(), n)
    gb = _map(occ, n, buckets=lb, static=static)
    for step in range(4):
        k = int(rng.integers(1, 300))
        xs = rng.integers(0, w, k).astype(np.int32)
        ys = rng.integers(0, h, k).astype(np.int32)
        vs = rng.integers(0, 2, k).astype(np.uint8)
        gb.update(xs, ys, vs)
        rm.update(xs, ys, vs)
        for i in range(k):
            occ[ys[i], xs[i]] = vs[i]
        x, y, th = _queries(rng, w, h, 8000)
        # plus rays from around the edited cells, in every direction: they read the refreshed buckets
        near = rng.integers(0, k, 8000)
        x = np.concatenate([x, (xs[near] + rng.uniform(-3, 4, 8000)).astype(np.float32)])
        y = np.concatenate([y, (ys[near] + rng.uniform(-3, 4, 8000)).astype(np.float32)])
        th = np.concatenate([th, rng.uniform(-math.pi, math.pi, 8000).astype(np.float32)])
        want = rm.cast(x, y, th, M, threads=4)
        got = gb.cast(_dev(x), _dev(y), _dev(th), M).cpu().numpy()
        assert (got == want).all(), f"step {step}: {(got != want).sum()} rays differ"
        # the lines rewritten in the edited bands, and the overflow count kept across the rewrites, equal a
        # fresh build's
        fresh = _map(occ.copy(), n, buckets=lb)
        assert gb.info()["bucket_overflow"] == fresh.info()["bucket_overflow"]
        assert (gb.bucket_lines() == fresh.bucket_lines()).all(), f"step {step}: bucket lines differ"
        fresh.close()


def test_bucket_plan_mixed_maps_equal_plain():
    """A batched plan over bucket and plain maps gives the plain per-filter weights bit for bit."""
    from paper_1705_01167_amd import cddt
    torch = _torch()
    rng = wl.rng_for(704, 0)
    M = 500
    filters, keep, plain, outs = [], [], [], []
    for f in range(6):
        side = int(rng.integers(200, 700))
        occ = wl.building_map(rng, side, side)
        n = int(rng.choice([108, 200, 360]))
        gm = _map(occ, n, buckets=(None if f % 2 else int(rng.choice([0, 6, 9]))))
        P = int(rng.integers(1, 3000))
        off = wl.ray_offsets(61)
        px, py, pth = wl.free_poses(rng, occ, P)
        obs, _ = wl.observations(rng, occ, off, M)
        table = wl.beam_table(M, wl.beam_params(rng))
        t = [_dev(px), _dev(py), _dev(pth), _dev(off), _dev(obs), _dev(table)]
        lw = gm.weight(*t, M)
        plain.append(lw.clone())
        out = torch.empty_like(lw)
        filters.append(cddt.make_filter(gm, *t, M, out))
        keep += [gm, t]
        outs.append(out)
    plan = cddt.Plan(filters, keepalive=keep)
    for tuning in ((8, 2, 8, 9), (4, 4, 4, 7), (16, 1, 16, 10), (2, 2, 2, 2), (8, 2, 8, 0)):
        plan.tuning = tuning
        for o in outs:
            o.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        for i, (got, want) in enumerate(zip(outs, plain)):
            assert torch.equal(got, want), f"tuning {tuning}: filter {i} differs"


@pytest.mark.parametrize("zp16", [False, True])
def test_bucket_casts_ragged_sizes(zp16):
    """Queued casts (4 x 64 rays per wave) at sizes around the tile and wave boundaries."""
    rng = wl.rng_for(705, int(zp16))
    occ = wl.building_map(rng, 300, 260)
    n = 108
    rm = oref.RefCDDT(occ, n, zp16=zp16)
    gb = _map(occ, n, buckets=6, zp16=zp16)
    for k in (1, 2, 63, 64, 65, 255, 256, 257, 1023, 4097):
        _say(f"bucket ragged zp16={zp16} n_rays={k}")
        x = rng.uniform(-2, 302, k).astype(np.float32)
        y = rng.uniform(-2, 262, k).astype(np.float32)
        th = rng.uniform(-7, 7, k).astype(np.float32)
        want = rm.cast(x, y, th, 400)
        got = gb.cast(_dev(x), _dev(y), _dev(th), 400).cpu().numpy()
        assert got.shape == want.shape and (got == want).all(), f"{k} rays"


@pytest.mark.parametrize("n,lb", [(8, 4), (64, None)])
def test_largest_map(n, lb):
    """The largest map (16384^2): with 8 bins and 2^4-cell buckets the 45-degree slice has the most
    buckets per band any map can have (1449); casts equal the oracle."""
    side = 16384
    rng = wl.rng_for(706, n)
    occ = np.zeros((side, side), np.uint8)
    occ[0, :] = occ[-1, :] = occ[:, 0] = occ[:, -1] = 1
    for _ in range(40):
        x0, y0 = int(rng.integers(1, side - 300)), int(rng.integers(1, side - 300))
        w, h = int(rng.integers(1, 300)), int(rng.integers(1, 300))
        occ[y0:y0 + h, x0:x0 + w] = 1
    _say(f"largest map n={n} buckets={lb}")
    rm = oref.RefCDDT(occ, n, threads=8)
    gm = _map(occ, n, buckets=lb)
    if lb is not None:
        info = gm.info()
        assert info["bucket_lines"] == info["rows"] * 1449
    k = 50000
    x = rng.uniform(0, side, k).astype(np.float32)
    y = rng.uniform(0, side, k).astype(np.float32)
    th = rng.uniform(-math.pi, math.pi, k).astype(np.float32)
    want = rm.cast(x, y, th, 65535, threads=8)
    got = gm.cast(_dev(x), _dev(y), _dev(th), 65535).cpu().numpy()
    assert (got == want).all(), f"{(got != want).sum()} rays differ"
    gm.close()
