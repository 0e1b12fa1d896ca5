"""Serving loop: results are the same alone and in the mix, under budget admission,
and every served log-weight equals the oracle's within 1e-5 * max(1, |L|)."""
import sys

import numpy as np
import pytest

from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _setup(seed=0, sides=(300, 500, 800), bins=(108, 200, 360), M=300, layouts=None):
    from paper_1705_01167_amd import cddt
    rng = wl.rng_for(501, seed)
    maps, offs, tabs, occs = [], [], [], []
    for f, (side, n) in enumerate(zip(sides, bins)):
        occ = wl.building_map(rng, side, side)
        maps.append(cddt.Map(_dev(occ), n, **(layouts[f] if layouts else {})))
        offs.append(wl.ray_offsets(61))
        tabs.append(_dev(wl.beam_table(M, wl.beam_params(rng))))
        occs.append(occ)
    return rng, maps, offs, tabs, occs, M


def _check_oracle(reqs, outs, maps, offs, tabs, occs, M, zp16=()):
    """Every served result against the plain C++ oracle's double log-sum (Sec. VI)."""
    refs = {}
    for out, (m, px, py, pth, obs) in zip(outs, reqs):
        if m not in refs:
            refs[m] = oref.RefCDDT(occs[m], maps[m].theta_bins, zp16=m in zp16)
        want = refs[m].weight(px, py, pth, offs[m], obs, tabs[m].cpu().numpy(), M)
        got = np.asarray(out, np.float64)
        assert np.isfinite(got).all()
        assert (np.abs(got - want) <= 1e-5 * np.maximum(1.0, np.abs(want))).all(), f"map {m}"
    for r in refs.values():
        r.close()


def _requests(rng, occs, M, k):
    reqs = []
    for i in range(k):
        m = i % len(occs)
        n = int(round(np.exp(rng.uniform(np.log(17), np.log(1639)))))
        px, py, pth = wl.free_poses(rng, occs[m], n)
        obs = rng.integers(0, M + 1, 61).astype(np.int32)
        reqs.append((m, px, py, pth, obs))
    return reqs


def test_alone_equals_mix_equals_plain():
    from paper_1705_01167_amd import cddt
    rng, maps, offs, tabs, occs, M = _setup()
    reqs = _requests(rng, occs, M, 120)
    srv = cddt.Server(maps, offs, tabs, [M] * 3, budget_bytes=8 << 20, n_lanes=4, max_batch=32)
    alone = []
    for (m, px, py, pth, obs) in reqs:
        alone.append(srv.wait(srv.submit(m, px, py, pth, obs)))
    ids = [srv.submit(*r) for r in reqs]          # all at once: batched, several lanes in flight
    mixed = [srv.wait(i) for i in ids]
    st = srv.stats()
    assert st["completed"] == 240 and st["rejected"] == 0
    assert st["batches"] < 240                     # requests really were batched together
    assert st["peak_bytes"] <= 8 << 20
    for a, b, (m, px, py, pth, obs) in zip(alone, mixed, reqs):
        assert a.tobytes() == b.tobytes()
        plain = maps[m].weight(_dev(px), _dev(py), _dev(pth), _dev(offs[m]), _dev(obs), tabs[m], M)
        assert plain.cpu().numpy().tobytes() == a.tobytes()
    for i in ids:
        s, d = srv.times(i)
        assert 0 <= s <= d
    srv.close()
    _check_oracle(reqs, mixed, maps, offs, tabs, occs, M)


def test_mixed_map_layouts_equal_plain():
    """Resident maps with the bucket index, with 16-bit lines and without the index:
    the server runs the persistent kernel built for 16-bit lines, and every result
    equals the plain call on its map."""
    from paper_1705_01167_amd import cddt
    layouts = [dict(buckets=6), dict(buckets=7, zp16=True), dict()]
    rng, maps, offs, tabs, occs, M = _setup(seed=3, layouts=layouts)
    reqs = _requests(rng, occs, M, 90)
    srv = cddt.Server(maps, offs, tabs, [M] * 3, budget_bytes=8 << 20, n_lanes=1, max_batch=32)
    ids = [srv.submit(*r) for r in reqs]
    got = [srv.wait(i) for i in ids]
    assert srv.stats()["completed"] == 90
    for a, (m, px, py, pth, obs) in zip(got, reqs):
        plain = maps[m].weight(_dev(px), _dev(py), _dev(pth), _dev(offs[m]), _dev(obs), tabs[m], M)
        assert plain.cpu().numpy().tobytes() == a.tobytes(), f"map {m} ({layouts[m]})"
    srv.close()
    _check_oracle(reqs, got, maps, offs, tabs, occs, M, zp16=(1,))


def test_replay_equals_submit():
    """Open-loop replay from the native thread gives the same results as submit; times are the schedule."""
    from paper_1705_01167_amd import cddt
    rng, maps, offs, tabs, occs, M = _setup(seed=3)
    reqs = _requests(rng, occs, M, 60)
    srv = cddt.Server(maps, offs, tabs, [M] * 3, budget_bytes=8 << 20, n_lanes=2, max_batch=16)
    ref = [srv.wait(srv.submit(*r)) for r in reqs]
    at = np.cumsum(np.full(len(reqs), 2e-4))
    ids = srv.replay(reqs, at)
    assert (ids >= 0).all()
    arrive = []
    replayed = []
    for rid, r in zip(ids.tolist(), ref):
        replayed.append(srv.wait(rid))
        assert replayed[-1].tobytes() == r.tobytes()
        s, d = srv.times(rid)
        assert s <= d
        arrive.append(s)
    gaps = np.diff(arrive)
    assert np.allclose(gaps, 2e-4, atol=1e-9)      # submit time is the scheduled arrival
    with pytest.raises(cddt.CddtError):
        srv.replay(reqs[:2], [1e-3, 0.0])           # decreasing offsets: refused, nothing submitted
    assert srv.stats()["submitted"] == 120
    srv.close()
    _check_oracle(reqs, replayed, maps, offs, tabs, occs, M)


def test_budget_admission_and_reject():
    from paper_1705_01167_amd import cddt
    rng, maps, offs, tabs, occs, M = _setup(seed=1, sides=(256,), bins=(108,))
    # each lane holds about 2 mid-size requests: many small batches, still exact
    srv = cddt.Server(maps, offs, tabs, [M], budget_bytes=2 * 64 * 1024, n_lanes=2, max_batch=64)
    reqs = _requests(rng, occs, M, 40)
    reqs = [r for r in reqs if r[1].size <= 1500]
    ids = [srv.submit(*r) for r in reqs]
    outs = [srv.wait(i) for i in ids]
    st = srv.stats()
    assert st["peak_bytes"] <= 2 * 64 * 1024 and st["batches"] >= len(reqs) // 8
    for o, (m, px, py, pth, obs) in zip(outs, reqs):
        plain = maps[m].weight(_dev(px), _dev(py), _dev(pth), _dev(offs[m]), _dev(obs), tabs[m], M)
        assert plain.cpu().numpy().tobytes() == o.tobytes()
    _check_oracle(reqs, outs, maps, offs, tabs, occs, M)
    big = wl.free_poses(rng, occs[0], 20000)
    with pytest.raises(cddt.CddtError) as e:
        srv.submit(0, *big, reqs[0][4])
    assert e.value.code == cddt.EBUSY
    assert srv.stats()["rejected"] == 1
    srv.close()


def test_poll_and_close_with_queue():
    from paper_1705_01167_amd import cddt
    rng, maps, offs, tabs, occs, M = _setup(seed=2, sides=(400,), bins=(200,))
    srv = cddt.Server(maps, offs, tabs, [M], budget_bytes=4 << 20, n_lanes=1, max_batch=4)
    reqs = _requests(rng, occs, M, 30)
    ids = [srv.submit(*r) for r in reqs]
    got = {}
    while len(got) < len(ids):
        for i in ids:
            if i not in got:
                r = srv.poll(i)
                if r is not None:
                    got[i] = r
    assert all(np.isfinite(v).all() for v in got.values())
    more = [srv.submit(*r) for r in reqs]   # left queued or in flight: close must still return
    srv.close()
