"""The 64-filter workload at full size in the other layouts bench.py measures
(`--buckets 7`, `--buckets none`, `--buckets 7 --zp16`: 16-bit bucket lines;
`--prune`: PCDDT with the 2^6-cell index), built and launched as bench.py does
them (graph replay, the 8,1,16,7 tuning): on filters spread over the map sizes,
every ray's range equals the oracle's reading of that layout (Sec. IV-B; for
16-bit lines Sec. IV-C's zero points at 1/8-cell bin centres; for PCDDT the
zero points some discrete state's cast returns) and every log-weight is within
1e-5 * max(1, |L|) of its double sum.  The pruned oracle casts from every
discrete state, so it is checked on the filters with the smallest maps.
"""
import sys

import numpy as np
import pytest

from oracle import ref as oref

pytestmark = pytest.mark.gpu

RTOL = 1e-5
TUNING = (8, 1, 16, 7)


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def _run(monkeypatch, buckets, zp16, prune, pick):
    import torch
    assert torch.cuda.is_available(), "GPU tests need a ROCm device"
    import bench
    from paper_1705_01167_amd import cddt
    monkeypatch.setattr(bench, "BUCKETS", buckets)
    monkeypatch.setattr(bench, "ZP16", zp16)
    monkeypatch.setattr(bench, "PRUNE", prune)
    specs, filters, keep, host, off_h, _ = bench.build_batched(64, with_ranges=True)
    stream = torch.cuda.Stream()
    plan = cddt.Plan(filters, stream=stream, keepalive=keep)
    plan.tuning = TUNING
    plan.capture(stream)
    for _ in range(2):
        plan.replay(stream)
    stream.synchronize()
    plan.close()
    chosen = pick(specs)
    for f in chosen:
        sp, h = specs[f], host[f]
        rg = keep[f][1]["ranges"].cpu().numpy()
        lw = keep[f][2].cpu().numpy().astype(np.float64)
        rm = oref.RefCDDT(h["occ"], h["n"], threads=oref.default_threads(), zp16=zp16, prune=prune)
        want_lw, want_rg = rm.weight(h["px"], h["py"], h["pth"], off_h, h["obs"], h["table"], bench.MAX_RANGE,
                                     threads=oref.default_threads(), want_ranges=True)
        rm.close()
        bad = int((rg != want_rg).sum())
        assert bad == 0, f"filter {f} (side {sp['side']}, n {h['n']}): {bad} ranges differ"
        assert (np.abs(lw - want_lw) <= RTOL * np.maximum(1.0, np.abs(want_lw))).all(), f"filter {f}: log-weights"
        _say(f"full variants: filter {f} (side {sp['side']}, {sp['particles']} particles) exact")
    for m, _, _ in keep:
        m.close()
    del keep, filters
    torch.cuda.empty_cache()
    return chosen


def _spread(specs, k=8):
    order = np.argsort([sp["side"] for sp in specs], kind="stable")
    return sorted(set(order[np.linspace(0, len(specs) - 1, k).round().astype(int)].tolist()))


def _smallest(specs, k=4):
    return sorted(np.argsort([sp["side"] for sp in specs], kind="stable")[:k].tolist())


@pytest.mark.timeout(900)
@pytest.mark.parametrize("buckets", [7, None])
def test_full_workload_bucket_widths_against_oracle(monkeypatch, buckets):
    _say(f"full variants: bucket index {buckets}")
    assert len(_run(monkeypatch, buckets, False, False, _spread)) == 8


@pytest.mark.timeout(900)
def test_full_workload_zp16_against_oracle(monkeypatch):
    _say("full variants: 16-bit bucket lines at 2^7 cells")
    assert len(_run(monkeypatch, 7, True, False, _spread)) == 8


@pytest.mark.timeout(900)
def test_full_workload_pcddt_against_oracle(monkeypatch):
    _say("full variants: PCDDT with the 2^6-cell index")
    assert len(_run(monkeypatch, 6, False, True, _smallest)) == 4
