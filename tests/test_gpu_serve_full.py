"""Serving at the size bench.py serves: the eight serving maps (sides 1000..4000,
theta bins from {108, 200, 360}, 2^7-cell bucket index), the resident server
with bench.py's tuning, slots and budget, and requests of 17..1639 particles
drawn as bench.py draws them.  Every served log-weight is within
1e-5 * max(1, |L|) of the oracle's double log-sum (Sec. VI beam model over the
Sec. IV-B/IV-C casts of the plain C++ CDDT), and requests served one at a time
give the same bits as the same requests served together.
"""
import sys

import numpy as np
import pytest

from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

sys.path.insert(0, __file__.rsplit("/", 1)[0])
from test_gpu_serve import _check_oracle  # noqa: E402


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def test_serving_maps_resident_against_oracle():
    import bench
    _say("serving full size: building the eight maps (2^7-cell bucket index)")
    maps, offs, tabs, pools, obs = bench.build_serving(7)
    occs = [wl.building_map(wl.rng_for(wl.SERVING, wl.S_MAP, i), side, side)
            for i, side in enumerate(bench.SERVE_SIDES)]
    reqs = bench.make_requests(96, 5, pools, obs)
    srv = bench.make_server(maps, offs, tabs, None, "r", 256 << 20)
    try:
        _say("serving full size: 8 requests one at a time")
        alone = [srv.wait(srv.submit(*r[:5])) for r in reqs[:8]]
        _say("serving full size: 96 requests at once from two submitting threads")
        ids = srv.replay([r[:5] for r in reqs], np.zeros(len(reqs)), threads=2)
        assert (ids >= 0).all()
        mixed = [srv.wait(int(i)) for i in ids]
        st = srv.stats()
    finally:
        srv.close()
    assert st["rejected"] == 0 and st["completed"] == 8 + len(reqs)
    for a, b in zip(alone, mixed[:8]):
        assert a.tobytes() == b.tobytes()
    _say("serving full size: every served log-weight against the oracle")
    _check_oracle([r[:5] for r in reqs], mixed, maps, offs, tabs, occs, bench.MAX_RANGE)
