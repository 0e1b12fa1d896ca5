"""The query-time suites (Sec. VI: casts from a uniformly spaced grid of states
and from uniformly random states) and the dense lookup-table comparator:

- casts of both suites equal the oracle's (the plain C++ CDDT, Sec. IV-B/IV-C
  reading) on plain, bucket-index and pruned maps, and the timed casts return
  the same ranges;
- the table built on the GPU equals the oracle's casts from every cell centre
  at every bin centre angle (for the pruned map too: pruning is exact from grid
  states, Sec. IV-C), and table lookups equal a gather from it by the query's
  cell and the oracle's binning;
- the cell-walk comparator equals the oracle's walk (exact.grid_traversal with
  the oracle's own sin and cos) query by query.
"""
import sys

import numpy as np
import pytest

from oracle import exact
from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

M = 200


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


MAPS = [("rect", 48, 40, 36), ("building", 90, 70, 108), ("random", 33, 29, 8)]
LAYOUTS = [dict(), dict(buckets=5), dict(static=True, prune=True)]


def _occ(kind, w, h, seed):
    rng = wl.rng_for(wl.SUITES, wl.S_MAP, seed)
    if kind == "rect":
        return wl.rect_map(rng, w, h, n_rects=6, side=(3, 9))
    if kind == "building":
        return wl.building_map(rng, w, h)
    return wl.random_map(rng, w, h, 0.15)


@pytest.mark.parametrize("mi", range(len(MAPS)))
def test_suites_and_table_against_oracle(mi):
    import torch
    from paper_1705_01167_amd import cddt
    kind, w, h, n = MAPS[mi]
    occ = _occ(kind, w, h, mi)
    rm = oref.RefCDDT(occ, n)
    gx, gy, gt = wl.grid_states(w, h, n, stride=1)
    rx, ry, rt = wl.random_states(wl.rng_for(wl.SUITES, wl.S_POSES, mi), w, h, 50000)
    want_grid = rm.cast(gx, gy, gt, M)
    want_rand = rm.cast(rx, ry, rt, M)
    want_lut = want_grid.reshape(n, h, w)   # every cell centre at every bin centre: the table's definition
    for lay in LAYOUTS:
        gm = cddt.Map(_dev(occ), n, **lay)
        for name, (x, y, t), want in (("grid", (gx, gy, gt), want_grid), ("random", (rx, ry, rt), want_rand)):
            if lay.get("prune") and name == "random":
                continue  # pruned maps answer exactly from grid states only
            got = gm.cast(_dev(x), _dev(y), _dev(t), M).cpu().numpy()
            assert (got == want).all(), f"{kind} {lay} {name}: {(got != want).sum()} casts differ"
            rg, ticks = gm.cast_timed(_dev(x), _dev(y), _dev(t), M)
            assert (rg.cpu().numpy() == want).all(), f"{kind} {lay} {name}: timed casts differ"
            assert (ticks.cpu().numpy() >= 0).all()
        lut = gm.lut(M)
        torch.cuda.synchronize()
        got_lut = lut.cpu().numpy().view(np.uint16)
        assert (got_lut == want_lut).all(), f"{kind} {lay}: {(got_lut != want_lut).sum()} table entries differ"
        gm.close()
    # table lookups: the query's cell and the oracle's bin; off-map, non-finite and huge angles give 0
    x = np.concatenate([rx, np.array([-0.1, w + 0.0, 1.5, 2.5], np.float32)])
    y = np.concatenate([ry, np.array([1.5, 1.5, np.nan, 2.5], np.float32)])
    t = np.concatenate([rt, np.array([0.3, 0.3, 0.3, 2e6], np.float32)])
    got, ticks = cddt.lut_cast(_dev(want_lut.astype(np.int16)), _dev(x), _dev(y), _dev(t), timed=True)
    got = got.cpu().numpy()
    want = np.zeros(x.size, np.int32)
    for q in range(x.size):
        if abs(t[q]) < 1e6 and 0 <= x[q] < w and 0 <= y[q] < h:
            want[q] = want_lut[exact.theta_bin(t[q], n), int(np.floor(y[q])), int(np.floor(x[q]))]
    assert (got == want).all(), f"{kind}: {(got != want).sum()} lookups differ"
    assert (ticks.cpu().numpy() >= 0).all()
    rm.close()
    _say(f"suites {kind} {w}x{h} n={n}: {gx.size} grid and {rx.size} random casts exact on {len(LAYOUTS)} layouts")


@pytest.mark.parametrize("mi", range(len(MAPS)))
def test_march_comparator_against_oracle(mi):
    from paper_1705_01167_amd import cddt
    kind, w, h, n = MAPS[mi]
    occ = _occ(kind, w, h, mi)
    gm = cddt.Map(_dev(occ), n)
    x, y, t = wl.random_states(wl.rng_for(wl.SUITES, wl.S_OBS, mi), w, h, 3000)
    gx, gy, gt = wl.grid_states(w, h, n, stride=max(1, w // 12))
    x = np.concatenate([x, gx, np.array([-1.0, 1.5, 1.5], np.float32)])
    y = np.concatenate([y, gy, np.array([1.5, 1.5, 1.5], np.float32)])
    t = np.concatenate([t, gt, np.array([0.0, np.inf, -3e6], np.float32)])
    got, ticks = gm.march(_dev(x), _dev(y), _dev(t), M, timed=True)
    got = got.cpu().numpy()
    want = np.array([oref.march_cast(occ, x[q], y[q], t[q], M) for q in range(x.size)], np.int32)
    bad = np.flatnonzero(got != want)
    assert bad.size == 0, f"{kind}: {bad.size} walks differ, first {[(x[q], y[q], t[q], got[q], want[q]) for q in bad[:3]]}"
    assert (ticks.cpu().numpy() >= 0).all()
    gm.close()
    _say(f"march {kind}: {x.size} walks exact")
