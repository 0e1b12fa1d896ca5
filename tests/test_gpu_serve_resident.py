"""Resident serving (one persistent kernel fed through a ring of slots):

- every result is bit-identical alone, in the mix, and to the plain call on its
  map, and within 1e-5 * max(1, |L|) of the oracle's double log-sum (Sec. VI);
- requests submitted while earlier ones are on the device are admitted into
  the running kernel (one launch serves them all);
- after the kernel leaves on an idle server, the next request launches it again;
- more requests than slots wait for slots; a request larger than a slot is
  refused; closing with work in flight or waiting returns.
"""
import sys
import time

import numpy as np
import pytest

from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_serve import _check_oracle, _dev, _requests, _setup  # noqa: E402

TUNING = (8, 2, 2, 7)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _server(maps, offs, tabs, M, slots=64, budget=64 << 20, tuning=TUNING):
    from paper_1705_01167_amd import cddt
    return cddt.Server(maps, offs, tabs, [M] * len(maps), budget_bytes=budget, n_lanes=1, max_batch=slots,
                       tuning=tuning, resident=True)


def _plain(maps, offs, tabs, M, r):
    m, px, py, pth, obs = r
    return maps[m].weight(_dev(px), _dev(py), _dev(pth), _dev(offs[m]), _dev(obs), tabs[m], M).cpu().numpy()


@pytest.mark.parametrize("tuning", [(8, 2, 2, 7), (4, 4, 1, 6), (16, 2, 2, 8), (2, 4, 1, 0)])
def test_resident_alone_equals_mix_equals_plain(tuning):
    rng, maps, offs, tabs, occs, M = _setup(seed=11)
    reqs = _requests(rng, occs, M, 100)
    srv = _server(maps, offs, tabs, M, slots=32, tuning=tuning)
    _say(f"resident {tuning}: one at a time")
    alone = [srv.wait(srv.submit(*r)) for r in reqs]
    _say(f"resident {tuning}: all at once")
    ids = [srv.submit(*r) for r in reqs]          # more requests than slots: some wait for a slot
    mixed = [srv.wait(i) for i in ids]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 200 and st["rejected"] == 0
    assert st["peak_bytes"] <= 64 << 20
    for a, b, r in zip(alone, mixed, reqs):
        assert a.tobytes() == b.tobytes()
        assert _plain(maps, offs, tabs, M, r).tobytes() == a.tobytes()
    _check_oracle(reqs, mixed, maps, offs, tabs, occs, M)


def test_resident_admits_while_running():
    """A second group submitted while the first is on the device is served by the
    same launch; results equal plain calls."""
    rng, maps, offs, tabs, occs, M = _setup(seed=12)
    first = _requests(rng, occs, M, 60)
    second = _requests(rng, occs, M, 60)
    srv = _server(maps, offs, tabs, M, slots=256)
    ids1 = [srv.submit(*r) for r in first]
    ids2 = [srv.submit(*r) for r in second]       # the kernel is running the first group by now
    got = [srv.wait(i) for i in ids1 + ids2]
    st = srv.stats()
    srv.close()
    _say(f"resident admission: {st}")
    assert st["completed"] == 120
    assert st["batches"] == 1                      # one kernel launch served both groups
    for a, r in zip(got, first + second):
        assert _plain(maps, offs, tabs, M, r).tobytes() == a.tobytes()


def test_resident_relaunch_after_idle():
    rng, maps, offs, tabs, occs, M = _setup(seed=13)
    reqs = _requests(rng, occs, M, 40)
    srv = _server(maps, offs, tabs, M)
    a = [srv.wait(srv.submit(*r)) for r in reqs[:20]]
    time.sleep(0.05)                               # the kernel leaves an idle server
    b = [srv.wait(srv.submit(*r)) for r in reqs[20:]]
    st = srv.stats()
    srv.close()
    assert st["completed"] == 40 and st["batches"] >= 2
    for x, r in zip(a + b, reqs):
        assert _plain(maps, offs, tabs, M, r).tobytes() == x.tobytes()


def test_resident_mixed_layouts_and_limits():
    from paper_1705_01167_amd import cddt
    layouts = [dict(buckets=6), dict(buckets=7, zp16=True), dict()]
    rng, maps, offs, tabs, occs, M = _setup(seed=14, layouts=layouts)
    reqs = _requests(rng, occs, M, 60)
    # slots of 16 KiB: 1,100 particles (18 KB of poses, observations and log-weights) do not fit
    srv = _server(maps, offs, tabs, M, slots=8, budget=8 * 16384)
    m0 = 2
    px, py, pth = wl.free_poses(rng, occs[m0], 1100)
    with pytest.raises(cddt.CddtError):
        srv.submit(m0, px, py, pth, reqs[0][4])
    small = [r for r in reqs if r[1].size <= 700][:30]
    ids = [srv.submit(*r) for r in small]
    got = [srv.wait(i) for i in ids]
    # an empty request finishes at once
    e = srv.submit(0, np.zeros(0, np.float32), np.zeros(0, np.float32), np.zeros(0, np.float32), reqs[0][4])
    assert srv.wait(e).size == 0
    st = srv.stats()
    srv.close()
    assert st["rejected"] == 1 and st["completed"] == len(small) + 1
    for a, r in zip(got, small):
        assert _plain(maps, offs, tabs, M, r).tobytes() == a.tobytes()
    _check_oracle(small, got, maps, offs, tabs, occs, M, zp16=(1,))


def test_resident_close_with_work():
    rng, maps, offs, tabs, occs, M = _setup(seed=15)
    reqs = _requests(rng, occs, M, 80)
    srv = _server(maps, offs, tabs, M, slots=4)
    for r in reqs:
        srv.submit(*r)
    srv.close()                                    # returns with requests in flight and waiting
    # the device is free again for plain work
    got = _plain(maps, offs, tabs, M, reqs[0])
    assert got.size == reqs[0][1].size


@pytest.mark.parametrize("resident", [True, False])
def test_replay_from_several_threads(resident):
    """Replay from three submitting threads (request i by thread i mod 3): every result equals the plain
    call on its map, and every recorded submit time is the request's scheduled arrival."""
    from paper_1705_01167_amd import cddt
    rng, maps, offs, tabs, occs, M = _setup(seed=16)
    reqs = _requests(rng, occs, M, 90)
    srv = cddt.Server(maps, offs, tabs, [M] * len(maps), budget_bytes=16 << 20, n_lanes=1 if resident else 2,
                      max_batch=64, tuning=TUNING, resident=resident)
    at = np.cumsum(np.full(len(reqs), 1e-4))
    ids = srv.replay(reqs, at, threads=3)
    assert (ids >= 0).all() and len(set(ids.tolist())) == len(reqs)
    t_first = None
    for rid, r, a in zip(ids.tolist(), reqs, at):
        got = srv.wait(rid)
        assert _plain(maps, offs, tabs, M, r).tobytes() == got.tobytes()
        s, d = srv.times(rid)
        t_first = s - a if t_first is None else t_first
        assert abs((s - a) - t_first) < 1e-9 and s <= d
    with pytest.raises(cddt.CddtError):
        srv.replay(reqs[:2], at[:2], threads=17)     # 1..16 threads
    st = srv.stats()
    srv.close()
    assert st["submitted"] == len(reqs) and st["completed"] == len(reqs)
