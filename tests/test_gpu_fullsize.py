"""Full-length parity at full size, against the oracle's stored samples
(tests/golden/make_oracle_samples.py runs only the FP64 CPU oracle):

  - D2Q9 4096^2 double shear layer, tau = 0.5001, 1000 steps, FP64 and FP32
    deviation storage, bulk correction off and on, compared at 4096 seeded
    nodes (normwise over the samples: 1e-12 FP64, 1e-5 FP32);
  - the first 32 domains of the batched shear-wave workload (512 domains,
    seed 2303), 2000 steps, run together in one pool (one persistent launch;
    and for FP64 two steps per launch, in 1000 launches and in one
    tile-ordered persistent launch): each equals the same domain run alone
    bitwise and matches the oracle at 64 seeded nodes;
  - all 512 domains of that workload in one persistent pool launch, in 1000
    two-step launches, and in one tile-ordered two-step launch, equal their
    single-domain runs bitwise.
"""
import os

import numpy as np
import pytest

from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden")
TOL = {"fp64": 1e-12, "fp32_dev": 1e-5}
GiB = 1 << 30


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


def _gold(name):
    path = os.path.join(GOLD, name)
    if not os.path.exists(path):
        pytest.skip(f"{name} not generated (tests/golden/make_oracle_samples.py)")
    return np.load(path, allow_pickle=False)


def rel_err(a, b):
    return float(np.max(np.abs(np.asarray(a) - np.asarray(b))) / np.max(np.abs(b)))


@pytest.fixture(scope="module")
def c2_fields():
    return workloads.double_shear_layer(4096)


@pytest.mark.parametrize("dtype", ["fp64", "fp32_dev"])
@pytest.mark.parametrize("corr", [False, True])
def test_c2_4096_full_steps_vs_oracle(c2_fields, dtype, corr):
    g = _gold("c2_double_shear_4096_1000.npz")
    key = "min" if corr else "off"
    assert int(g[f"bad_{key}"]) == 0
    lbm = _lbm()
    rho0, u0 = c2_fields
    with lbm.Domain(rho0, u0, float(g["tau"]), dtype=dtype, bulk_correction=corr) as d:
        d.step(int(g["steps"]))
        rho, u, diag = d.moments()
    xs, ys = g["x"], g["y"]
    er = rel_err(rho[ys, xs], g[f"rho_{key}"])
    eu = rel_err(u[:, ys, xs], g[f"u_{key}"])
    print(f"[parity] D2Q9 4096^2 double shear 1000 steps {dtype} corr={corr} (4096 samples): "
          f"rel err rho {er:.3e}  u {eu:.3e}", flush=True)
    assert diag["steps"] == 1000
    assert er < TOL[dtype] and eu < TOL[dtype]


def _alone(r0, u0, tau, steps, dtype):
    lbm = _lbm()
    with lbm.Domain(r0, u0, tau, dtype=dtype) as d:
        d.step(steps)
        rho, u, _ = d.moments()
    return rho, u


# pool tunings of the batched runs: one persistent launch per run (one step per
# grid-barrier phase), two steps per launch (the serving default), and every
# two-step iteration in one tile-ordered persistent launch
C4_TUNINGS = {"persistent": dict(persistent=1), "two_step": dict(tile_x=64, tile_y=4, time_block=2),
              "tile_ordered": dict(tile_x=64, tile_y=4, time_block=2, persistent=1)}
C4_LAUNCHES = {"persistent": lambda steps: 1, "two_step": lambda steps: steps // 2, "tile_ordered": lambda steps: 1}


@pytest.mark.parametrize("dtype,form", [("fp64", "persistent"), ("fp32_dev", "persistent"), ("fp64", "two_step"),
                                        ("fp64", "tile_ordered")])
def test_c4_subset_full_steps_vs_oracle_and_alone(dtype, form):
    g = _gold("c4_subset_2000.npz")
    count, steps = int(g["count"]), int(g["steps"])
    specs = workloads.batch_domains(count=512, seed=2303)[:count]
    lbm = _lbm()
    fields = [workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"]) for sp in specs]
    worst = [0.0, 0.0]
    with lbm.Pool(GiB, max_slots=count, tuning=lbm.make_pool_tuning(**C4_TUNINGS[form])) as pool:
        slots = [pool.admit(r, u, sp["tau"], steps, dtype=dtype) for (r, u), sp in zip(fields, specs)]
        pool.run(steps)
        assert set(pool.poll()) == set(slots)
        # the form that ran: one launch per run, or one per two steps
        assert pool.stats()["launches"] == C4_LAUNCHES[form](steps)
        for k, (s, sp, (r0, u0)) in enumerate(zip(slots, specs, fields)):
            assert int(g[f"bad_{k}"]) == 0
            rho, u, _ = pool.moments(s)
            ra, ua = _alone(r0, u0, sp["tau"], steps, dtype)
            assert np.array_equal(rho, ra) and np.array_equal(u, ua), k
            xs, ys = g[f"x_{k}"], g[f"y_{k}"]
            er = rel_err(rho[ys, xs], g[f"rho_{k}"])
            eu = rel_err(u[:, ys, xs], g[f"u_{k}"])
            worst = [max(worst[0], er), max(worst[1], eu)]
            assert er < TOL[dtype] and eu < TOL[dtype], (k, sp, er, eu)
    print(f"[parity] batched shear waves, 32 domains x 2000 steps {dtype} ({form}): worst rel err rho {worst[0]:.3e}  "
          f"u {worst[1]:.3e}", flush=True)


@pytest.fixture(scope="module")
def c4_alone_fp32():
    """All 512 batched domains run alone (FP32 deviation storage, 2000 steps)."""
    specs = workloads.batch_domains(count=512, seed=2303)
    out = []
    for sp in specs:
        r0, u0 = workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"])
        out.append(_alone(r0, u0, sp["tau"], 2000, "fp32_dev"))
    return specs, out


@pytest.mark.parametrize("form", ["persistent", "two_step", "tile_ordered"])
def test_c4_all_512_pool_equals_alone_bitwise(c4_alone_fp32, form):
    lbm = _lbm()
    specs, alone = c4_alone_fp32
    steps = 2000
    with lbm.Pool(4 * GiB, max_slots=512, tuning=lbm.make_pool_tuning(**C4_TUNINGS[form])) as pool:
        slots = []
        for sp in specs:
            r0, u0 = workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"])
            slots.append(pool.admit(r0, u0, sp["tau"], steps, dtype="fp32_dev"))
        pool.run(steps)
        assert set(pool.poll()) == set(slots)
        assert pool.stats()["launches"] == C4_LAUNCHES[form](steps)
        for s, sp, (ra, ua) in zip(slots, specs, alone):
            rho, u, d = pool.moments(s)
            assert d["steps"] == steps
            assert np.array_equal(rho, ra) and np.array_equal(u, ua), sp
