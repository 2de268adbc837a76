"""Checkpoint and restart (lbm_state_bytes / lbm_save_state / lbm_load_state):
a run saved at step k, loaded into a fresh domain of the same configuration and
tuning, and continued, must give the bits of the uninterrupted run, for both
storage types, every lattice, the vector kernels, and a z-slab (whose saved
state includes its halo planes).  Also: the step count is restored, the
domain flag is cleared on load, and mismatched sizes are refused."""
import numpy as np
import pytest

from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


CASES = [  # (fields, dtype, correction, tuning kwargs)
    (lambda: workloads.taylor_green_2d(64), "fp64", False, None),
    (lambda: workloads.random_field((33, 70), seed=11, umax=0.1), "fp32_dev", True, None),
    (lambda: workloads.random_field((7, 9, 13), seed=12, umax=0.1), "fp32_dev", False, None),
    (lambda: workloads.random_field((6, 5, 256), seed=13, umax=0.1), "fp32_dev", True,
     dict(block_x=64, nodes_per_thread=4)),
    (lambda: workloads.random_field((4, 6, 128), seed=14, umax=0.1), "fp64", False,
     dict(block_x=64, nodes_per_thread=2)),
    (lambda: workloads.random_field((100,), seed=15, umax=0.1), "fp64", True, None),
    # multi-step launches: the saved state is the same stored buffer
    (lambda: workloads.random_field((24, 192), seed=19, umax=0.1), "fp32_dev", True, dict(time_block=2)),
    (lambda: workloads.random_field((3000,), seed=20, umax=0.1), "fp32_dev", False, dict(time_block=8)),
]


@pytest.mark.parametrize("case", range(len(CASES)))
def test_restart_continues_bitwise(case):
    lbm = _lbm()
    make, dtype, corr, tun = CASES[case]
    rho0, u0 = make()
    tuning = lbm.make_tuning(**tun) if tun else None
    kw = dict(dtype=dtype, bulk_correction=corr, tuning=tuning)
    # the fresh domain starts from other fields: everything it keeps must come from the state
    rho1, u1 = workloads.random_field(rho0.shape, seed=99, umax=0.05)
    with lbm.Domain(rho0, u0, 0.57, **kw) as a, lbm.Domain(rho1, u1, 0.57, **kw) as b:
        a.step(37)  # an odd count: the saved state lies in the second buffer
        state, steps = a.save_state()
        assert steps == 37 and state.numel() == lbm.lbm_state_bytes(a.handle)
        a.step(45)
        b.step(3)  # b's current buffer differs from a's at save time
        b.load_state(state, steps)
        b.step(45)
        ra, ua, da = a.moments()
        rb, ub, db = b.moments()
        assert da["steps"] == db["steps"] == 82
        assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
        assert np.array_equal(a.populations(), b.populations())


def test_restart_of_a_z_slab():
    """One slab that is its own neighbour (periodic in z): the restarted copy
    reloads the halo planes with the state and continues bitwise."""
    import torch
    lbm = _lbm()
    rho0, u0 = workloads.random_field((6, 10, 18), seed=16, umax=0.1)
    slabs = [lbm.Domain(rho0, u0, 0.6, dtype="fp32_dev", z_halo=True) for _ in range(2)]
    try:
        nb = slabs[0].halo_bytes()
        lo = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        hi = torch.empty(nb, dtype=torch.uint8, device="cuda:0")

        def advance(s, n):
            for _ in range(n):
                s.halo_pack(lo, hi)
                s.halo_unpack(hi, lo)
                s.step(1)

        a, b = slabs
        advance(a, 9)
        a.halo_pack(lo, hi)
        a.halo_unpack(hi, lo)  # the halo planes are filled when the state is saved
        state, steps = a.save_state()
        for _ in range(11):
            a.step(1)
            a.halo_pack(lo, hi)
            a.halo_unpack(hi, lo)
        b.load_state(state, steps)
        for _ in range(11):
            b.step(1)
            b.halo_pack(lo, hi)
            b.halo_unpack(hi, lo)
        assert a.moments()[2]["steps"] == b.moments()[2]["steps"] == 20
        assert np.array_equal(a.populations(), b.populations())
    finally:
        for s in slabs:
            s.close()


def test_load_clears_the_domain_flag_and_checks_sizes():
    import torch
    lbm = _lbm()
    rho0, u0 = workloads.random_field((16, 16), seed=17, umax=0.05)
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64") as good:
        state, steps = good.save_state()
        # a rough field near |u| = 1 at tau -> 1/2 leaves the equilibrium's domain within 20 steps
        bad_r, bad_u = workloads.random_field((16, 16), seed=70, umax=0.99, rho_lo=0.3, rho_hi=2.0)
        with lbm.Domain(bad_r, bad_u, 0.5001, dtype="fp64") as bad:
            bad.step(20)
            with pytest.raises(lbm.LBMDomainError):
                bad.save_state()
            bad.load_state(state, steps)  # same shape and storage; its own tau stays
            assert bad.moments()[2]["steps"] == 0
            assert np.array_equal(good.populations(), bad.populations())
        short = state[:-8]
        with pytest.raises(lbm.LBMError):
            good.load_state(short, 0)
        with pytest.raises(lbm.LBMError):
            good.load_state(state, -1)
        with lbm.Domain(*workloads.random_field((16, 16), seed=18, umax=0.05), 0.6, dtype="fp32_dev") as other:
            with pytest.raises(lbm.LBMError):  # another storage type: another size
                other.load_state(state, steps)
        assert torch.cuda.is_available()
