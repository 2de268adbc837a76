"""GPU test of the autotuner: it times candidate pool tunings, returns one that
runs, caches it, and the tuned pool gives the same results as the default."""
import numpy as np
import pytest

from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def test_autotune_small_batch(tmp_path):
    from paper_2303_08163_amd import autotune, lbm
    specs = workloads.batch_domains(count=12, seed=7, lo=32, hi=160)
    doms = [(9, (s["nx"], s["ny"]), "fp32_dev") for s in specs]
    cache = str(tmp_path / "tune.json")
    cands = [dict(tile_x=64, tile_y=4, persistent=0), dict(tile_x=32, tile_y=8, persistent=1),
             dict(tile_x=128, tile_y=2, persistent=1)]
    best, rep = autotune.tune_pool(doms, steps=5, cands=cands, cache_path=cache)
    assert best in cands and not rep["cached"] and len(rep["times"]) == 3 and rep["failed"] == []
    best2, rep2 = autotune.tune_pool(doms, steps=5, cands=cands, cache_path=cache)
    assert best2 == best and rep2["cached"]
    results = []
    for tun in (lbm.make_pool_tuning(**best), None):
        with lbm.Pool(1 << 28, max_slots=16, tuning=tun) as pool:
            slots = []
            for s in specs:
                r0, u0 = workloads.shear_wave(s["nx"], s["ny"], s["amp"])
                slots.append(pool.admit(r0, u0, s["tau"], 30))
            pool.run(30)
            pool.poll()
            results.append([pool.moments(k)[:2] for k in slots])
    for (ra, ua), (rb, ub) in zip(*results):
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub)


def test_default_candidates_all_run(tmp_path):
    """Every candidate of the default set runs on a mix that reaches each launch
    form: a D2Q9 FP32 class large enough for two steps per launch (so that the
    two-step and tile-ordered candidates take those forms), ragged small D2Q9
    slots in the same class, and a D3Q27 class (one step per launch, or the
    grid-barrier form for the persistent candidates).  None is refused or fails."""
    from paper_2303_08163_amd import autotune
    doms = [(9, (2048, 2100), "fp32_dev"), (9, (100, 37), "fp32_dev"), (9, (513, 65), "fp32_dev"),
            (27, (40, 33, 21), "fp32_dev")]
    cands = autotune.candidates()
    assert any(c.get("persistent") and c.get("time_block") == 2 for c in cands)
    best, rep = autotune.tune_pool(doms, steps=6, cands=cands, cache_path=str(tmp_path / "tune.json"))
    assert rep["failed"] == [], rep["failed"]
    assert len(rep["times"]) == len(cands) and best in cands
