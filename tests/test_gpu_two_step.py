"""Several LBGK steps per launch (lbm_tuning.time_block): two on D2Q9, and
2, 4 or 8 on D1Q3.  On D2Q9 (time_block = 2) the
intermediate state stays in LDS, and every node runs the same collision code
as the one-step kernels, so results must be bitwise those of the default
one-step path -- for both storage types, with and without the correction,
on ragged row counts, degenerate grids (one or two rows, a single column
tile), odd step counts (ending with one one-step launch) and graph replays.
The domain flag must rise exactly when it rises on the one-step path; the
oracle closes the loop at FP64 tolerance."""
import numpy as np
import pytest

import oracle
from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


CASES = [  # (ny, nx), dtype, correction, time_rows, step chunks
    ((64, 64), "fp32_dev", False, 0, (1, 2, 7, 100)),
    ((100, 192), "fp64", True, 7, (65, 3)),
    ((1, 128), "fp32_dev", True, 1, (6, 1)),
    ((2, 64), "fp64", False, 0, (5,)),
    ((3, 512), "fp32_dev", False, 2, (4, 64)),
    ((37, 256), "fp32_dev", True, 37, (9,)),
    ((48, 320), "fp64", False, 5, (2, 2, 131)),
    # ragged widths: the last tile of each row is partial
    ((30, 100), "fp32_dev", True, 0, (3, 64)),
    ((17, 1000), "fp64", True, 4, (7,)),
    ((5, 65), "fp32_dev", False, 2, (2, 65)),
    ((64, 777), "fp64", False, 9, (4, 33)),
    ((40, 1500), "fp32_dev", True, 0, (11,)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_two_step_equals_one_step_bitwise(case):
    lbm = _lbm()
    shape, dtype, corr, rows, chunks = CASES[case]
    rho0, u0 = workloads.random_field(shape, seed=40 + case, umax=0.1)
    two = lbm.make_tuning(time_block=2, time_rows=rows)
    with lbm.Domain(rho0, u0, 0.55, dtype=dtype, bulk_correction=corr, tuning=two) as a, \
            lbm.Domain(rho0, u0, 0.55, dtype=dtype, bulk_correction=corr) as b:
        done = 0
        for n in chunks:
            a.step(n)
            b.step(n)
            done += n
            ra, ua, da = a.moments()
            rb, ub, db = b.moments()
            assert da["steps"] == db["steps"] == done
            assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (shape, done)
        assert np.array_equal(a.populations(), b.populations())


def test_two_step_matches_oracle():
    lbm = _lbm()
    rho0, u0 = workloads.taylor_green_2d(64, u0=0.05)
    for corr in (False, True):
        r_ref, u_ref, bad = oracle.run(rho0, u0, 0.53, 50, corr="min" if corr else "off")
        assert bad == 0
        with lbm.Domain(rho0, u0, 0.53, dtype="fp64", bulk_correction=corr,
                        tuning=lbm.make_tuning(time_block=2)) as d:
            d.step(50)
            rho, u, diag = d.moments()
        assert np.max(np.abs(rho - r_ref)) / np.max(np.abs(r_ref)) < 1e-12
        assert np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)) < 1e-12


def test_two_step_domain_flag_as_one_step():
    """The flag is the OR over every node of both steps, halo duplicates
    included: it must rise in the same call as on the one-step path."""
    lbm = _lbm()
    for seed in range(70, 74):
        rho0, u0 = workloads.random_field((16, 64), seed=seed, umax=0.99, rho_lo=0.3, rho_hi=2.0)
        with lbm.Domain(rho0, u0, 0.5001, dtype="fp64", tuning=lbm.make_tuning(time_block=2)) as a, \
                lbm.Domain(rho0, u0, 0.5001, dtype="fp64") as b:
            for n in (1, 2, 3, 6, 10):
                a.step(n)
                b.step(n)
                fa = a.moments(fields=False, raise_on_domain=False)[2]["domain_error"]
                fb = b.moments(fields=False, raise_on_domain=False)[2]["domain_error"]
                assert fa == fb, (seed, n)


def test_two_step_ragged_large_bitwise():
    """A large ragged width (4000^2, 1024-column tiles with a partial last
    one of 928), where two steps per launch are the default."""
    lbm = _lbm()
    rho0, u0 = workloads.random_field((4000, 4000), seed=51, umax=0.1)
    with lbm.Domain(rho0, u0, 0.51, dtype="fp32_dev") as a:
        a.step(3)
        fa = a.populations()
    with lbm.Domain(rho0, u0, 0.51, dtype="fp32_dev", tuning=lbm.make_tuning(time_block=1)) as b:
        b.step(3)
        assert np.array_equal(fa, b.populations())


@pytest.mark.parametrize("dtype", ["fp32_dev", "fp64"])
def test_two_step_full_size_bitwise(dtype):
    """D2Q9 4096^2 (the large 2-D workload), 4 steps with the default
    two-step kernel (columns of 1024 for FP32 storage, 128 for FP64) against
    one step per launch."""
    lbm = _lbm()
    rho0, u0 = workloads.random_field((4096, 4096), seed=50, umax=0.1)
    with lbm.Domain(rho0, u0, 0.51, dtype=dtype) as a:
        info = a.launch_info()
        assert info["kernel"] == "two_step", info
        assert info["time_cols"] == (1024 if dtype == "fp32_dev" else 128), info
        a.step(4)
        fa = a.populations()
    with lbm.Domain(rho0, u0, 0.51, dtype=dtype, tuning=lbm.make_tuning(time_block=1)) as b:
        b.step(4)
        assert np.array_equal(fa, b.populations())


def test_two_step_fp32_ragged_matches_oracle():
    """The two-step kernel with FP32 deviation storage against the FP64
    oracle on a ragged width (165: column tiles of 128, the last of 37) and
    ragged rows (45 in tiles of 8), with and without the correction, 60
    steps."""
    lbm = _lbm()
    rho0, u0 = workloads.random_field((45, 165), seed=77, umax=0.1)
    for corr in (False, True):
        r_ref, u_ref, bad = oracle.run(rho0, u0, 0.53, 60, corr="min" if corr else "off")
        assert bad == 0
        with lbm.Domain(rho0, u0, 0.53, dtype="fp32_dev", bulk_correction=corr,
                        tuning=lbm.make_tuning(time_block=2, time_rows=8)) as d:
            info = d.launch_info()
            assert info["kernel"] == "two_step" and info["time_cols"] == 128, info
            d.step(60)
            rho, u, diag = d.moments()
        er = np.max(np.abs(rho - r_ref)) / np.max(np.abs(r_ref))
        eu = np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref))
        print(f"[parity] D2Q9 165x45 two-step FP32 corr={corr} 60 steps: rel err rho {er:.3e} u {eu:.3e}", flush=True)
        assert er < 1e-5 and eu < 1e-5


D1Q3_CASES = [  # nx, dtype, correction, K, step chunks
    (1032, "fp32_dev", False, 2, (1, 2, 7, 64)),
    (1500, "fp32_dev", True, 4, (3, 70)),
    (4096, "fp64", False, 8, (8, 9, 100)),
    (520, "fp64", True, 8, (17,)),
    (1 << 20, "fp32_dev", True, 8, (40,)),
    (5000, "fp64", True, 4, (66,)),
    # short rows: tx = nx - 8 owned nodes per workgroup, two workgroups
    (16, "fp64", True, 8, (8, 3, 64)),
    (17, "fp32_dev", False, 8, (9, 16)),
    (64, "fp32_dev", True, 8, (10, 10, 70)),
    (100, "fp64", False, 2, (5, 64)),
    (255, "fp32_dev", True, 4, (13,)),
]


@pytest.mark.parametrize("case", range(len(D1Q3_CASES)))
def test_d1q3_multi_step_equals_one_step_bitwise(case):
    """K steps per launch on D1Q3 (LDS segments with K nodes of halo): bitwise
    the one-step path, on ragged lengths, the smallest allowed length, graph
    replays (>= 64 steps) and counts that leave a remainder."""
    lbm = _lbm()
    nx, dtype, corr, K, chunks = D1Q3_CASES[case]
    rho0, u0 = workloads.random_field((nx,), seed=60 + case, umax=0.1)
    with lbm.Domain(rho0, u0, 0.55, dtype=dtype, bulk_correction=corr,
                    tuning=lbm.make_tuning(time_block=K)) as a, \
            lbm.Domain(rho0, u0, 0.55, dtype=dtype, bulk_correction=corr,
                       tuning=lbm.make_tuning(time_block=1)) as b:
        done = 0
        for n in chunks:
            a.step(n)
            b.step(n)
            done += n
            ra, ua, da = a.moments()
            rb, ub, db = b.moments()
            assert da["steps"] == db["steps"] == done
            assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (nx, K, done)
        assert np.array_equal(a.populations(), b.populations())


def test_d1q3_multi_step_matches_oracle_and_flags():
    lbm = _lbm()
    rho0, u0 = workloads.pressure_wave(2048, 1e-3, 0.1)
    r_ref, u_ref, bad = oracle.run(rho0, u0, 0.6, 48, corr="min")
    assert bad == 0
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64", bulk_correction=True, tuning=lbm.make_tuning(time_block=8)) as d:
        d.step(48)
        rho, u, _ = d.moments()
    assert np.max(np.abs(rho - r_ref)) / np.max(np.abs(r_ref)) < 1e-12
    assert np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)) < 1e-12
    for seed in range(80, 83):
        rho0, u0 = workloads.random_field((2048,), seed=seed, umax=0.99, rho_lo=0.3, rho_hi=2.0)
        with lbm.Domain(rho0, u0, 0.5001, dtype="fp64", tuning=lbm.make_tuning(time_block=4)) as a, \
                lbm.Domain(rho0, u0, 0.5001, dtype="fp64", tuning=lbm.make_tuning(time_block=1)) as b:
            for n in (1, 4, 5, 8):
                a.step(n)
                b.step(n)
                fa = a.moments(fields=False, raise_on_domain=False)[2]["domain_error"]
                fb = b.moments(fields=False, raise_on_domain=False)[2]["domain_error"]
                assert fa == fb, (seed, n)


@pytest.mark.parametrize("eq", ["poly2", "product"])
def test_multi_step_polynomial_equilibria_bitwise(eq):
    """The polynomial and product-form equilibria take the same multi-step
    kernels: two steps on D2Q9, four on D1Q3, bitwise one step per launch."""
    lbm = _lbm()
    for shape, K, dtype in (((36, 256), 2, "fp32_dev"), ((40, 192), 2, "fp64"), ((3000,), 4, "fp32_dev"),
                            ((1100,), 4, "fp64")):
        rho0, u0 = workloads.random_field(shape, seed=90, umax=0.08)
        kw = dict(dtype=dtype, bulk_correction=True, equilibrium=eq)
        with lbm.Domain(rho0, u0, 0.56, tuning=lbm.make_tuning(time_block=K), **kw) as a, \
                lbm.Domain(rho0, u0, 0.56, tuning=lbm.make_tuning(time_block=1), **kw) as b:
            a.step(70)
            b.step(70)
            assert np.array_equal(a.populations(), b.populations()), (eq, shape)
