"""The query-time suites at the size bench.py runs them (the 2000^2 floor at 200
bins and the 1000^2 room map at 108 bins, 500 x 500 grid positions at every bin
centre angle, and as many uniformly random states; Sec. VI), checked on sampled
outputs that the oracle computes one by one:

- casts on the plain map and with the 2^7-cell bucket index (untimed and
  timed, which agree everywhere) equal the oracle's casts (the plain C++ CDDT,
  Sec. IV-B/IV-C reading) on a seeded sample of each suite;
- the dense lookup table holds, at every sampled grid state, the oracle's cast
  from that cell centre at that bin centre angle, and table lookups of sampled
  random states equal the table entry of the query's cell and the oracle's bin;
- the cell walk equals the oracle's walk on a sample of random states.
"""
import sys

import numpy as np
import pytest

from oracle import exact
from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

SAMPLE = 1 << 17
WALK_SAMPLE = 1500


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _bins(t, n):
    """The oracle's theta bin (exact.theta_bin), for many angles: float32 product, float32 add, floor, mod n."""
    u = (t.astype(np.float32) * np.float32(exact.bin_scale(n))).astype(np.float32) + np.float32(0.5)
    return np.floor(u.astype(np.float64)).astype(np.int64) % n


@pytest.mark.parametrize("mi", [0, 1])
def test_suites_full_size_sampled_against_oracle(mi):
    import torch
    import bench
    from paper_1705_01167_amd import cddt
    name, side, n = bench.SUITE_MAPS[mi]
    M = bench.MAX_RANGE
    seed_map = (wl.FLOOR, wl.S_MAP) if side == 2000 else (wl.SUITES, wl.S_MAP)
    occ = wl.building_map(wl.rng_for(*seed_map), side, side)
    stride = side // bench.SUITE_POSITIONS
    suites = {"grid": wl.grid_states(side, side, n, stride),
              "random": wl.random_states(wl.rng_for(wl.SUITES, wl.S_POSES, mi), side, side,
                                         bench.SUITE_POSITIONS * bench.SUITE_POSITIONS * n)}
    rm = oref.RefCDDT(occ, n)
    rng = np.random.default_rng(1000 + mi)
    sel = {k: np.sort(rng.choice(v[0].size, SAMPLE, replace=False)) for k, v in suites.items()}
    want = {k: rm.cast(v[0][sel[k]], v[1][sel[k]], v[2][sel[k]], M) for k, v in suites.items()}
    rm.close()
    dev = {k: tuple(_dev(a) for a in v) for k, v in suites.items()}
    for lay in ({}, {"buckets": 7}):
        gm = cddt.Map(_dev(occ), n, **lay)
        for k, (x, y, t) in dev.items():
            got = gm.cast(x, y, t, M)
            rg_t, ticks = gm.cast_timed(x, y, t, M)
            assert torch.equal(got, rg_t), f"{name} {lay} {k}: timed casts differ from untimed"
            g = got.cpu().numpy()[sel[k]]
            assert (g == want[k]).all(), f"{name} {lay} {k}: {(g != want[k]).sum()} of {SAMPLE} sampled casts differ"
        gm.close()
        _say(f"suites full {name} {lay}: {2 * SAMPLE} sampled casts exact")
    gm = cddt.Map(_dev(occ), n)
    lut = gm.lut(M)  # (bins, rows, columns) of 16-bit ranges
    torch.cuda.synchronize()
    # grid query q is bin k = q // P^2, row stride * ((q // P) % P), column stride * (q % P), P = positions per axis
    q = sel["grid"]
    pos = bench.SUITE_POSITIONS
    ent = lut[_dev(q // (pos * pos)), _dev(stride * ((q // pos) % pos)), _dev(stride * (q % pos))]
    ent = ent.cpu().numpy().view(np.uint16).astype(np.int32)
    assert (ent == want["grid"]).all(), f"{name}: {(ent != want['grid']).sum()} sampled table entries differ"
    rx, ry, rt = suites["random"]
    got = cddt.lut_cast(lut, dev["random"][0], dev["random"][1], dev["random"][2]).cpu().numpy()[sel["random"]]
    s = sel["random"]
    gat = lut[_dev(_bins(rt[s], n)), _dev(np.floor(ry[s]).astype(np.int64)), _dev(np.floor(rx[s]).astype(np.int64))]
    gat = gat.cpu().numpy().view(np.uint16).astype(np.int32)
    assert (got == gat).all(), f"{name}: {(got != gat).sum()} sampled lookups differ"
    del lut
    w = s[:WALK_SAMPLE]
    walk = gm.march(_dev(rx[w]), _dev(ry[w]), _dev(rt[w]), M).cpu().numpy()
    ref = np.array([oref.march_cast(occ, rx[q], ry[q], rt[q], M) for q in w], np.int32)
    assert (walk == ref).all(), f"{name}: {(walk != ref).sum()} of {w.size} walks differ"
    gm.close()
    _say(f"suites full {name}: table entries, lookups and {w.size} walks agree")
