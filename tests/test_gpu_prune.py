"""PCDDT (pruned static CDDT) on the GPU against the oracle's PCDDT reading.

The pruned structure must equal the oracle's bit for bit (export), casts
anywhere must equal the oracle's PCDDT casts, casts from the grid states must
equal the unpruned structure, and log-weights stay within 1e-5.  Also with the
bucket index on the pruned bands, after updates (rebuild and prune), and
inside a batched plan.
"""
import math
import sys

import numpy as np
import pytest

from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _map(occ, n, **kw):
    from paper_1705_01167_amd import cddt
    return cddt.Map(_dev(occ), n, **kw)


def _states(occ, n):
    jj, ii = np.nonzero(occ == 0)
    x = np.repeat(ii.astype(np.float32) + np.float32(0.5), n)
    y = np.repeat(jj.astype(np.float32) + np.float32(0.5), n)
    th = (2.0 * math.pi * np.tile(np.arange(n), ii.size) / n).astype(np.float32)
    return x, y, th


def _queries(rng, w, h, k):
    x = rng.uniform(-2, w + 2, k).astype(np.float32)
    y = rng.uniform(-2, h + 2, k).astype(np.float32)
    th = rng.uniform(-40, 40, k).astype(np.float32)
    x[4:100] = np.floor(x[4:100]) + np.float32(0.5)
    return x, y, th


def _same_export(gm, rm):
    for a, b in zip(gm.export(), rm.export()):
        assert a.shape == b.shape and (a == b).all()


@pytest.mark.parametrize("seed", range(8))
def test_prune_tiny_maps(seed):
    rng = wl.rng_for(961, seed)
    w, h = int(rng.integers(1, 80)), int(rng.integers(1, 80))
    occ = wl.random_map(rng, w, h, float(rng.uniform(0.0, 0.6)))
    n = int(rng.choice([2, 8, 36, 108, 200]))
    full = seed % 4 == 3
    lb = [None, 0, 5, 9][seed % 4]
    M = int(rng.choice([0, 7, 100, 65535]))
    _say(f"prune tiny seed={seed} {w}x{h} n={n} full={full} buckets={lb} M={M}")
    rm = oref.RefCDDT(occ, n, full_map=full, prune=True)
    gm = _map(occ, n, full_map=full, prune=True, buckets=lb)
    _same_export(gm, rm)
    x, y, th = _queries(rng, w, h, 20000)
    got = gm.cast(_dev(x), _dev(y), _dev(th), M).cpu().numpy()
    assert (got == rm.cast(x, y, th, M, threads=4)).all()
    if (occ == 0).any():
        sx, sy, sth = _states(occ, n)
        full_rm = oref.RefCDDT(occ, n, full_map=full)
        got = gm.cast(_dev(sx), _dev(sy), _dev(sth), 65535).cpu().numpy()
        assert (got == full_rm.cast(sx, sy, sth, 65535, threads=4)).all()


@pytest.mark.parametrize("lb", [None, 7])
def test_prune_floor_2000(lb):
    occ = wl.building_map(wl.rng_for(wl.FLOOR, wl.S_MAP), 2000, 2000)
    n, M = 200, 500
    rm = oref.RefCDDT(occ, n, threads=8, prune=True)
    gm = _map(occ, n, prune=True, buckets=lb)
    info = gm.info()
    _say(f"prune floor buckets={lb}: {info['zero_points']} zero points")
    _same_export(gm, rm)
    off = wl.ray_offsets(61)
    px, py, pth = wl.free_poses(wl.rng_for(wl.FLOOR, wl.S_POSES), occ, 2500)
    table = wl.beam_table(M, wl.beam_params(wl.rng_for(wl.FLOOR, wl.S_TABLE)))
    obs, _ = wl.observations(wl.rng_for(wl.FLOOR, wl.S_OBS), occ, off, M)
    ref_lw, ref_r = rm.weight(px, py, pth, off, obs, table, M, threads=8, want_ranges=True)
    lw, rr = gm.weight(_dev(px), _dev(py), _dev(pth), _dev(off), _dev(obs), _dev(table), M, ranges=True)
    assert (rr.cpu().numpy() == ref_r).all()
    lw = lw.cpu().numpy().astype(np.float64)
    assert (np.abs(lw - ref_lw) <= 1e-5 * np.maximum(1.0, np.abs(ref_lw))).all()


@pytest.mark.parametrize("seed", range(3))
def test_prune_updates_rebuild(seed):
    rng = wl.rng_for(962, seed)
    w, h = int(rng.integers(30, 120)), int(rng.integers(30, 120))
    occ = wl.random_map(rng, w, h, 0.15)
    n = int(rng.choice([36, 108]))
    lb = [None, 6, 0][seed]
    _say(f"prune updates seed={seed} {w}x{h} n={n} buckets={lb}")
    rm = oref.RefCDDT(occ.copy(), n, prune=True)
    gm = _map(occ, n, prune=True, buckets=lb)
    for step in range(3):
        k = int(rng.integers(1, 200))
        xs = rng.integers(0, w, k).astype(np.int32)
        ys = rng.integers(0, h, k).astype(np.int32)
        vs = rng.integers(0, 2, k).astype(np.uint8)
        gm.update(xs, ys, vs)
        rm.update(xs, ys, vs)
        _same_export(gm, rm)
        x, y, th = _queries(rng, w, h, 5000)
        got = gm.cast(_dev(x), _dev(y), _dev(th), 300).cpu().numpy()
        assert (got == rm.cast(x, y, th, 300, threads=4)).all(), f"step {step}"


def test_prune_in_plan_equals_plain():
    from paper_1705_01167_amd import cddt
    import torch
    rng = wl.rng_for(963, 0)
    M = 500
    filters, keep, plain, outs = [], [], [], []
    for f in range(4):
        side = int(rng.integers(150, 500))
        occ = wl.building_map(rng, side, side)
        n = int(rng.choice([108, 200]))
        gm = _map(occ, n, prune=(f % 2 == 0), buckets=(7 if f < 2 else None))
        P = int(rng.integers(1, 2000))
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
    for tuning in ((8, 2, 8, 9), (4, 2, 8, 7), (8, 2, 8, 0)):
        plan.tuning = tuning
        for o in outs:
            o.fill_(float("nan"))
        plan.run()
        torch.cuda.synchronize()
        for i, (got, want) in enumerate(zip(outs, plain)):
            assert torch.equal(got, want), f"tuning {tuning}: filter {i}"
