"""cddt_batch_weight: the batched step in one call, without a plan.

Filters on room/corridor maps of uneven size and layout (plain bands, the
bucket index, 16-bit lines, pruned), uneven particle counts (empty filters
included) and more filters than one descriptor chunk carries:

- every range equals the oracle's cast (Sec. IV-B/IV-C reading) and every
  log-weight is within 1e-5 * max(1, |L|) of the oracle's double sum (Sec. VI),
  except the 16-bit maps, whose ranges follow the oracle's 16-bit reading;
- the log-weights equal a plan's over the same filters and tuning bit for bit,
  at several tunings and with no tuning (the recorded one);
- a call recorded into a graph replays to the same bits, with eager work and
  synchronisations between the replays;
- a second call with fewer filters and particles on the same stream is right.
"""
import sys

import numpy as np
import pytest

from oracle import ref as oref
from paper_1705_01167_amd import workloads as wl

pytestmark = pytest.mark.gpu

M = 300
RTOL = 1e-5


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _dev(a):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    return torch.from_numpy(np.ascontiguousarray(a)).cuda()


def _filters(seed, n_filters, max_side, ranges=True):
    """n_filters filters; layouts cycle through plain, bucket, 16-bit and pruned maps."""
    import torch
    from paper_1705_01167_amd import cddt
    rng = wl.rng_for(seed, 0)
    off_h = wl.ray_offsets(61)
    off = _dev(off_h)
    layouts = [dict(), dict(buckets=6), dict(buckets=7, zp16=True), dict(static=True, prune=True)]
    out = []
    for f in range(n_filters):
        kw = layouts[f % len(layouts)]
        w = int(rng.integers(64, max_side))
        h = int(rng.integers(64, max_side))
        n = int(rng.choice([36, 108, 200]))
        occ = wl.building_map(rng, w, h)
        gm = cddt.Map(_dev(occ), n, **kw)
        npart = 0 if f == 3 else int(rng.integers(1, 400))
        px, py, pth = wl.free_poses(rng, occ, npart)
        obs, _ = wl.observations(rng, occ, off_h, M)
        table = wl.beam_table(M, wl.beam_params(rng))
        d = dict(px=_dev(px), py=_dev(py), pth=_dev(pth), obs=_dev(obs), table=_dev(table))
        lw = torch.full((npart,), float("nan"), dtype=torch.float32, device="cuda")
        rg = torch.full((npart, 61), -1, dtype=torch.int32, device="cuda") if ranges else None
        flt = cddt.make_filter(gm, d["px"], d["py"], d["pth"], off, d["obs"], d["table"], M, lw, ranges=rg)
        out.append(dict(flt=flt, gm=gm, d=d, lw=lw, rg=rg, occ=occ, n=n, kw=kw,
                        host=(px, py, pth, obs, table), off_h=off_h, off=off))
    return out


def _oracle_check(fs, tag):
    for i, f in enumerate(fs):
        px, py, pth, obs, table = f["host"]
        kw = f["kw"]
        rm = oref.RefCDDT(f["occ"], f["n"], prune=bool(kw.get("prune")), zp16=bool(kw.get("zp16")))
        want_lw, want_rg = rm.weight(px, py, pth, f["off_h"], obs, table, M, want_ranges=True)
        rm.close()
        if f["rg"] is not None:
            got_rg = f["rg"].cpu().numpy()
            bad = int((got_rg != want_rg).sum())
            assert bad == 0, f"{tag}: filter {i} ({kw}): {bad} ranges differ from the oracle"
        got = f["lw"].cpu().numpy().astype(np.float64)
        assert np.isfinite(got).all()
        assert (np.abs(got - want_lw) <= RTOL * np.maximum(1.0, np.abs(want_lw))).all(), f"{tag}: filter {i}"


def _clear(fs):
    import torch
    for f in fs:
        f["lw"].fill_(float("nan"))
        if f["rg"] is not None:
            f["rg"].fill_(-1)
    torch.cuda.synchronize()


def _close(fs):
    for f in fs:
        f["gm"].close()


def test_batch_weight_equals_oracle_and_plan():
    import torch
    from paper_1705_01167_amd import cddt
    fs = _filters(511, 26, 320)  # two descriptor chunks
    flts = [f["flt"] for f in fs]
    stream = torch.cuda.Stream()
    keep = [(f["d"], f["lw"], f["rg"], f["off"]) for f in fs]
    for t in [(8, 2, 8, 7), (4, 4, 4, 8), (2, 4, 8, 2), (1, 4, 8, 0), None]:
        _clear(fs)
        cddt.batch_weight(flts, tuning=t, stream=stream)
        stream.synchronize()
        _say(f"one call: tuning {t}")
        _oracle_check(fs, f"one call, tuning {t}")
        got = [f["lw"].cpu().numpy().copy() for f in fs]
        _clear(fs)
        plan = cddt.Plan(flts, tuning=t, stream=stream, keepalive=keep)
        plan.run(stream)
        stream.synchronize()
        plan.close()
        for i, f in enumerate(fs):
            assert f["lw"].cpu().numpy().tobytes() == got[i].tobytes(), f"tuning {t}: filter {i} one call != plan"
    # a second, smaller call on the same stream: fewer filters, fewer particles
    small = _filters(512, 5, 200)
    _clear(small)
    cddt.batch_weight([f["flt"] for f in small], tuning=(8, 2, 8, 7), stream=stream)
    stream.synchronize()
    _oracle_check(small, "second, smaller call")
    _close(small)
    _close(fs)


def test_batch_weight_uses_recorded_tuning():
    import torch
    from paper_1705_01167_amd import cddt
    fs = _filters(513, 6, 256, ranges=False)
    flts = [f["flt"] for f in fs]
    t = (16, 2, 4, 8)
    cddt.tuning_cache_put(flts, t)
    assert cddt.tuning_cache_get(flts) == (t, True)
    stream = torch.cuda.Stream()
    cddt.batch_weight(flts, stream=stream)
    stream.synchronize()
    _oracle_check(fs, "recorded tuning")
    _close(fs)


def test_batch_weight_graph_replays():
    import torch
    from paper_1705_01167_amd import cddt
    fs = _filters(514, 9, 256)
    flts = [f["flt"] for f in fs]
    stream = torch.cuda.Stream()
    # the workspace grows outside capture first
    cddt.batch_weight(flts, tuning=(8, 2, 8, 7), stream=stream)
    stream.synchronize()
    eager = [f["lw"].cpu().numpy().copy() for f in fs]
    eager_rg = [f["rg"].cpu().numpy().copy() for f in fs]
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g, stream=stream):
        cddt.batch_weight(flts, tuning=(8, 2, 8, 7), stream=stream)
    for rep in range(3):
        _clear(fs)
        # eager work between replays (the one-call path on the same stream)
        with torch.cuda.stream(stream):
            g.replay()
        stream.synchronize()
        for i, f in enumerate(fs):
            assert f["lw"].cpu().numpy().tobytes() == eager[i].tobytes(), f"replay {rep}: filter {i}"
            assert (f["rg"].cpu().numpy() == eager_rg[i]).all(), f"replay {rep}: filter {i} ranges"
        cddt.batch_weight(flts[:3], tuning=(4, 4, 4, 8), stream=stream)
        stream.synchronize()
    _oracle_check(fs, "graph replays")
    _close(fs)
