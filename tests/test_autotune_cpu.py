"""Host logic of the pool autotuner: candidates that raise are reported, not
hidden, and the fastest remaining one is chosen and cached."""
import pytest

from paper_2303_08163_amd import autotune, lbm


def test_failed_candidates_are_reported(monkeypatch, tmp_path):
    cands = [dict(tile_x=64, tile_y=4, persistent=0), dict(tile_x=64, tile_y=4, persistent=1),
             dict(tile_x=128, tile_y=2, persistent=0), dict(tile_x=7, tile_y=1, persistent=0)]
    speed = {(64, 4, 0): 2e-3, (128, 2, 0): 1e-3}

    def fake_time(domains, c, steps=20, warmup=3):
        if c["persistent"]:
            raise lbm.LBMError(lbm.LBM_EDEVICE, "lbm_pool_poll", "a persistent launch's grid barrier timed out")
        if c["tile_x"] == 7:
            raise ValueError("tuning rejected")
        return speed[c["tile_x"], c["tile_y"], c["persistent"]]

    monkeypatch.setattr(autotune, "time_tuning", fake_time)
    monkeypatch.setattr(autotune, "_device_key", lambda: "test-device")
    doms = [(9, (40, 50), "fp32_dev")]
    cache = str(tmp_path / "tune.json")
    best, rep = autotune.tune_pool(doms, cands=cands, cache_path=cache)
    assert best == cands[2]
    assert [t for t, _ in rep["times"]] == [1.0, 2.0]
    assert [c for c, _ in rep["failed"]] == [cands[1], cands[3]]
    assert "grid barrier timed out" in rep["failed"][0][1]
    best2, rep2 = autotune.tune_pool(doms, cands=cands, cache_path=cache)
    assert best2 == best and rep2["cached"]


def test_all_candidates_failing_raises(monkeypatch):
    def fail(domains, c, steps=20, warmup=3):
        raise ValueError("rejected")

    monkeypatch.setattr(autotune, "time_tuning", fail)
    monkeypatch.setattr(autotune, "_device_key", lambda: "test-device")
    with pytest.raises(RuntimeError):
        autotune.tune_pool([(9, (40, 50), "fp64")], cands=[dict(tile_x=64, tile_y=4, persistent=0)], cache_path=None)


def test_candidate_sets():
    default = autotune.candidates()
    # persistent by default: only the tile-ordered two-step form (no grid barrier)
    assert default and all(c["persistent"] == 0 or c.get("time_block") == 2 for c in default)
    ordered = [c for c in default if c["persistent"] == 1]
    assert ordered and sorted(c["time_rows"] for c in ordered) == [0, 32]
    both = autotune.candidates(persistent=True)
    two = [c for c in default if c.get("time_block") == 2]  # no grid-barrier variant of these
    assert two and len(both) == 2 * len(default) - len(two)
    assert sorted(map(str, (c for c in both if c["persistent"] == 0 or c.get("time_block") == 2))) == \
        sorted(map(str, default))


def test_custom_candidates_do_not_share_the_default_cache(monkeypatch, tmp_path):
    calls = []

    def fake_time(domains, c, steps=20, warmup=3):
        calls.append(c)
        return 1e-3 if c["tile_x"] == 128 else 2e-3

    monkeypatch.setattr(autotune, "time_tuning", fake_time)
    monkeypatch.setattr(autotune, "_device_key", lambda: "test-device")
    cache = str(tmp_path / "tune.json")
    doms = [(9, (40, 50), "fp32_dev")]
    only64 = [dict(tile_x=64, tile_y=4, persistent=0)]
    best, _ = autotune.tune_pool(doms, cands=only64, cache_path=cache)
    assert best == only64[0]
    best2, rep2 = autotune.tune_pool(doms, cache_path=cache)  # default set: timed afresh
    assert not rep2["cached"] and best2["tile_x"] == 128
