"""Host logic of the autotuner: candidate sets per path, cache keys per
architecture, path and precision, the disk cache, and the plans it returns.
Plans and timings are replaced by fakes, so nothing here touches a GPU."""
import json

import pytest

from paper_1110_4874_amd import autotune, sht


class FakePlan:
    built = []

    def __init__(self, L, nside, eps, **kw):
        self.L, self.nside, self.eps, self.kw = L, nside, eps, kw
        FakePlan.built.append(self)

    def close(self):
        pass


def fake_time(plan, nmaps, *, steps=5, path=sht.PATH_AUTO, precision=sht.PREC_FP64, **_):
    # brute: fastest at 2 rings per lane, 512 threads; butterfly: rho 4 in
    # FP64, rho 2 in FP32
    kw = plan.kw
    if path == sht.PATH_BRUTE:
        return abs(kw["rings_per_lane"] - 2) + abs(kw["ring_threads"] - 512) / 256 + 1.0
    target = 4.0 if precision == sht.PREC_FP64 else 2.0
    return abs(kw["rho"] - target) + 0.5


@pytest.fixture
def fakes(monkeypatch):
    FakePlan.built = []
    monkeypatch.setattr(autotune.sht, "Plan", FakePlan)
    monkeypatch.setattr(autotune, "time_synthesis", fake_time)
    monkeypatch.setattr(autotune, "_cache", {})
    return FakePlan


def test_keys_name_arch_path_and_precision():
    k64 = autotune._key(255, 128, 4, 1e-12, sht.PATH_BUTTERFLY, sht.PREC_FP64)
    k32 = autotune._key(255, 128, 4, 1e-12, sht.PATH_BUTTERFLY, sht.PREC_FP32)
    kb = autotune._key(255, 128, 4, 0.0, sht.PATH_BRUTE, sht.PREC_FP64)
    assert k64 != k32 and k64 != kb
    assert k64.startswith(autotune.arch() + "/butterfly/fp64/")
    assert autotune.arch() == "none"  # no GPU in the CPU suite


def test_resolve_rules():
    assert autotune._resolve(0.0, sht.PATH_AUTO, sht.PREC_FP32) == (sht.PATH_BRUTE, sht.PREC_FP64)
    assert autotune._resolve(1e-12, sht.PATH_AUTO, sht.PREC_FP32) == (sht.PATH_BUTTERFLY, sht.PREC_FP32)
    with pytest.raises(ValueError):
        autotune._resolve(0.0, sht.PATH_BUTTERFLY, sht.PREC_FP64)
    with pytest.raises(ValueError):
        autotune._resolve(0.0, sht.PATH_INTERP, sht.PREC_FP64)


def test_brute_sweep_picks_the_fastest_shape(fakes):
    best = autotune.tune(127, 64, 4)
    assert {k: best[k] for k in ("rings_per_lane", "ring_threads")} == {"rings_per_lane": 2, "ring_threads": 512}
    assert len(fakes.built) == len(autotune.RINGS_PER_LANE) * len(autotune.RING_THREADS)
    assert all(p.eps == 0.0 for p in fakes.built)
    # a second call is served from the process cache
    autotune.tune(127, 64, 4)
    assert len(fakes.built) == 9


def test_butterfly_sweeps_rho_per_precision_with_the_brute_ring_shape(fakes):
    b64 = autotune.tune(255, 128, 4, 1e-12, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP64)
    n_after_64 = len(fakes.built)
    b32 = autotune.tune(255, 128, 4, 1e-12, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32)
    assert b64["rho"] == 4.0 and b32["rho"] == 2.0
    for b in (b64, b32):
        assert (b["rings_per_lane"], b["ring_threads"]) == (2, 512)
    # brute sweep once (shared by both precisions), then the rho values
    assert n_after_64 == 9 + len(autotune.BF_RHO)
    assert len(fakes.built) == 9 + 2 * len(autotune.BF_RHO)
    bf = [p for p in fakes.built if p.eps > 0]
    assert all(p.kw.get("store_fp32") for p in bf[len(autotune.BF_RHO):])  # FP32 candidates hold FP32 copies
    assert not any(p.kw.get("store_fp32") for p in bf[:len(autotune.BF_RHO)])


def test_disk_cache_round_trip(fakes, tmp_path, monkeypatch):
    f = tmp_path / "tune.json"
    best = autotune.tune(127, 64, 2, 1e-12, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32, cache_file=str(f))
    disk = json.load(open(f))
    assert set(disk) == {autotune._key(127, 64, 2, 1e-12, sht.PATH_BUTTERFLY, sht.PREC_FP32),
                         autotune._key(127, 64, 2, 0.0, sht.PATH_BRUTE, sht.PREC_FP64)}
    # a fresh process (empty memory cache) reads the file and times nothing
    monkeypatch.setattr(autotune, "_cache", {})
    n = len(fakes.built)
    again = autotune.tune(127, 64, 2, 1e-12, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32, cache_file=str(f))
    assert again == json.loads(json.dumps(best)) and len(fakes.built) == n


def test_tuned_plan_carries_the_knobs(fakes):
    p = autotune.tuned_plan(255, 128, 4, 1e-12, path=sht.PATH_BUTTERFLY, precision=sht.PREC_FP32)
    assert p.eps == 1e-12 and p.kw["rho"] == 2.0 and p.kw["store_fp32"] is True
    assert (p.kw["rings_per_lane"], p.kw["ring_threads"]) == (2, 512)
    q = autotune.tuned_plan(255, 128, 4, plan_eps=1e-10, plan_kw={"store_transpose": True})
    assert q.eps == 1e-10 and "rho" not in q.kw and q.kw["store_transpose"] is True
