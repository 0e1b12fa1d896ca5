"""A plan over maps that an update re-lays (static maps, pruned maps): the plan
calls take the moved band arrays into their descriptors, so runs, graph
replays and plain runs after the update equal the oracle on the new grid."""
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


def test_plan_after_relayout():
    import torch
    from paper_1705_01167_amd import cddt
    rng = wl.rng_for(408, 0)
    M, n = 300, 108
    off_h = wl.ray_offsets(61)
    off = _dev(off_h)
    layouts = [dict(static=True), dict(prune=True), dict(static=True, buckets=6)]
    occs, maps, host, filters, keep = [], [], [], [], []
    for f, kw in enumerate(layouts):
        occ = wl.building_map(rng, 260 + 40 * f, 240)
        gm = cddt.Map(_dev(occ), n, **kw)
        px, py, pth = wl.free_poses(rng, occ, 700 + 300 * f)
        obs, _ = wl.observations(rng, occ, off_h, M)
        table = wl.beam_table(M, wl.beam_params(rng))
        d = dict(px=_dev(px), py=_dev(py), pth=_dev(pth), obs=_dev(obs), table=_dev(table))
        lw = torch.zeros(px.size, dtype=torch.float32, device="cuda")
        rg = torch.zeros((px.size, 61), dtype=torch.int32, device="cuda")
        filters.append(cddt.make_filter(gm, d["px"], d["py"], d["pth"], off, d["obs"], d["table"], M, lw,
                                        ranges=rg))
        occs.append(occ)
        maps.append(gm)
        keep.append((d, lw, rg))
        host.append((px, py, pth, obs, table))
    stream = torch.cuda.Stream()
    plan = cddt.Plan(filters, tuning=(8, 4, 2, 7), stream=stream, keepalive=keep)

    def check(tag):
        stream.synchronize()
        for f, (kw, (px, py, pth, obs, table)) in enumerate(zip(layouts, host)):
            rm = oref.RefCDDT(occs[f], n, prune=bool(kw.get("prune")))
            want_lw, want_rg = rm.weight(px, py, pth, off_h, obs, table, M, want_ranges=True)
            rm.close()
            got_rg = keep[f][2].cpu().numpy()
            assert (got_rg == want_rg).all(), f"{tag}: filter {f} ({kw}) ranges"
            got = keep[f][1].cpu().numpy().astype(np.float64)
            assert (np.abs(got - want_lw) <= 1e-5 * np.maximum(1.0, np.abs(want_lw))).all(), f"{tag}: filter {f}"

    def clear():
        for _, lw, rg in keep:
            lw.fill_(float("nan"))
            rg.fill_(-1)
        torch.cuda.synchronize()

    plan.run(stream)
    check("before the update")
    plan.capture(stream)
    for step in range(2):
        before = [gm.info()["rebuilds"] for gm in maps]
        for f, gm in enumerate(maps):
            # a new wall segment: static bands have no slack, so the structure is re-laid
            j = int(rng.integers(20, 200))
            xs = np.arange(30, 90, dtype=np.int32)
            ys = np.full(xs.size, j, np.int32)
            vs = np.ones(xs.size, np.uint8)
            with torch.cuda.stream(stream):
                gm.update(xs, ys, vs, stream=stream)
            wl.apply_ops(occs[f], xs, ys, vs)
        rebuilt = [gm.info()["rebuilds"] > b for gm, b in zip(maps, before)]
        _say(f"plan after update {step}: re-laid {rebuilt}")
        assert rebuilt[0] and rebuilt[2]
        clear()
        plan.replay(stream)
        check(f"replay after update {step}")
        clear()
        plan.run(stream)
        check(f"run after update {step}")
        clear()
        plan.run_plain(stream)
        check(f"plain after update {step}")
    plan.close()
