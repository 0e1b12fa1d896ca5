"""Autotuner host logic (CPU only): it times every tuning in its grid on the
plan, skips tunings the library refuses, keeps the fastest after a
confirmation pass, and caches the choice under the plan signature."""
import json

import pytest

from paper_1705_01167_amd import cddt, tune


class FakePlan:
    """Stands in for cddt.Plan: a fixed cost per tuning, EINVAL for some."""

    def __init__(self, best, refused=()):
        self.best = best
        self.refused = set(refused)
        self.calls = 0
        self.tuning = None

    def time(self, t, reps=3, stream=None):
        self.calls += 1
        if t in self.refused:
            raise cddt.CddtError(cddt.EINVAL, "tuning outside the kernel's limits")
        return 1.0 + sum(abs(a - b) for a, b in zip(t, self.best)) * 0.01


@pytest.fixture
def cache_file(tmp_path, monkeypatch):
    p = tmp_path / "tuning.json"
    monkeypatch.setenv("CDDT_TUNE_CACHE", str(p))
    return p


def test_picks_fastest_skips_refused_and_caches(cache_file):
    best = (8, 2, 8, 7)
    refused = {(8, 2, 8, 8), (16, 8, 16, 10)}
    plan = FakePlan(best, refused)
    sig = tune.signature(64, 315690, [108, 200, 360, 360], "MI355X", buckets=6)
    got, ms, table = tune.autotune(plan, sig)
    assert got == best and plan.tuning == best and ms == 1.0
    grid = len(tune.SPACE_PPT) * len(tune.SPACE_WAVES) * len(tune.SPACE_BLOCKS) * len(tune.SPACE_K)
    assert len(table) == grid - len(refused)
    assert all(t not in refused for _, t in table)
    assert table == sorted(table)
    stored = json.loads(cache_file.read_text())
    assert stored[sig] == {"tuning": list(best), "ms": 1.0}
    # a second run with the same signature uses the cache and times nothing
    plan2 = FakePlan((1, 1, 1, 0))
    got2, ms2, table2 = tune.autotune(plan2, sig)
    assert got2 == best and plan2.tuning == best and plan2.calls == 0 and table2 == []
    # without the cache it sweeps again
    got3, _, _ = tune.autotune(plan2, sig, use_cache=False)
    assert got3 == (1, 1, 1, 0) and plan2.calls > 0


def test_other_errors_propagate(cache_file):
    class Broken(FakePlan):
        def time(self, t, reps=3, stream=None):
            raise cddt.CddtError(cddt.EDEVICE, "device failure")

    with pytest.raises(cddt.CddtError):
        tune.autotune(Broken((1, 1, 1, 0)), "sig", use_cache=False)


def test_signature_separates_layouts_and_shapes():
    base = dict(n_filters=64, total_particles=315690, theta_bins=[108, 200, 360], device_name="MI355X")
    s6 = tune.signature(**base, buckets=6)
    assert s6 != tune.signature(**base, buckets=7)
    assert s6 != tune.signature(**base, buckets=None)
    assert s6 != tune.signature(**base, buckets="6z16")
    assert s6 != tune.signature(**{**base, "n_filters": 32}, buckets=6)
    # the particle total is bucketed by powers of two; the theta-bin set is order free
    assert s6 == tune.signature(**{**base, "total_particles": 315000}, buckets=6)
    assert s6 == tune.signature(**{**base, "theta_bins": [360, 108, 200, 200]}, buckets=6)
