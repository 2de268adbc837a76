"""GPU tests of the pool (batching and serving): every slot's result equals the
same domain run alone, bitwise, whatever the mix, the admission time, the
launch form (one launch per step or one persistent cooperative launch) and the
tile shape; admission limits; failure isolation; and oracle parity."""
import numpy as np
import pytest

import oracle
from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu

GiB = 1 << 30


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


def alone(rho0, u0, tau, steps, dtype, corr):
    lbm = _lbm()
    with lbm.Domain(rho0, u0, tau, dtype=dtype, bulk_correction=corr) as d:
        d.step(steps)
        rho, u, diag = d.moments(raise_on_domain=False)
        f = d.populations()
    return rho, u, diag, f


MIX = [  # (init fields, tau, steps, dtype, correction)
    (lambda: workloads.taylor_green_2d(48, u0=0.08), 0.52, 37, "fp32_dev", False),
    (lambda: workloads.random_field((33, 70), seed=1, umax=0.2), 0.6, 20, "fp64", True),
    (lambda: workloads.taylor_green_3d(16, u0=0.07), 0.5005, 29, "fp32_dev", True),
    (lambda: workloads.shear_wave(96, 130, 0.05), 0.51, 50, "fp32_dev", False),
    (lambda: workloads.random_field((9, 11, 13), seed=2, umax=0.2), 0.7, 13, "fp64", False),
    (lambda: workloads.random_field((5, 300), seed=3, umax=0.3), 0.55, 1, "fp32_dev", True),
    (lambda: workloads.shear_wave(40, 40, 0.1, nz=24), 0.58, 0, "fp32_dev", False),
]


@pytest.fixture(scope="module")
def alone_results():
    out = []
    for make, tau, steps, dtype, corr in MIX:
        rho0, u0 = make()
        out.append((rho0, u0, alone(rho0, u0, tau, steps, dtype, corr)))
    return out


@pytest.mark.parametrize("persistent", [0, 1])
@pytest.mark.parametrize("tile", [(64, 4), (32, 2), (256, 1), ("flat", 64, 4), ("flat", 64, 1), ("fit", 64, 4),
                                  ("fit", 64, 2), ("fit-planes", 64, 4), ("two", 64, 4)])
@pytest.mark.parametrize("chunk", [1000, 7])
def test_pool_mix_equals_alone_bitwise(alone_results, persistent, tile, chunk):
    lbm = _lbm()
    if tile[0] == "two":
        # every class here is below the two-step size threshold, so the tuning
        # falls back to one step per launch (persistent: the grid-barrier form)
        tun = lbm.make_pool_tuning(tile[1], tile[2], persistent, time_block=2)
    elif tile[0] == "flat":
        tun = lbm.make_pool_tuning(tile[1], tile[2], persistent, flat=1)
    elif tile[0] in ("fit", "fit-planes"):
        layout = lbm.LBM_LAYOUT_PLANES if tile[0] == "fit-planes" else 0
        tun = lbm.make_pool_tuning(tile[1], tile[2], persistent, layout=layout, row_fit=1)
    else:
        tun = lbm.make_pool_tuning(tile[0], tile[1], persistent)
    with lbm.Pool(GiB // 4, max_slots=16, tuning=tun) as pool:
        slots = []
        for (make, tau, steps, dtype, corr), (rho0, u0, _) in zip(MIX, alone_results):
            slots.append(pool.admit(rho0, u0, tau, steps, dtype=dtype, bulk_correction=corr))
        finished = set()
        for _ in range(200):
            pool.run(chunk)
            finished |= set(pool.poll())
            if len(finished) == len(slots):
                break
        assert finished == set(slots)
        for s, (make, tau, steps, dtype, corr), (_, _, (rho, u, diag, f)) in zip(slots, MIX, alone_results):
            r2, u2, d2 = pool.moments(s, raise_on_domain=False)
            assert d2["steps"] == steps
            assert np.array_equal(r2, rho) and np.array_equal(u2, u)
            assert np.array_equal(pool.populations(s), f)
        assert pool.stats()["launches"] > 0


def test_pool_continuous_admission_equals_alone(alone_results):
    """Requests admitted while others are mid-run, released as they finish."""
    lbm = _lbm()
    with lbm.Pool(GiB // 4, max_slots=3) as pool:
        pending = list(range(len(MIX)))
        active = {}
        checked = 0
        for _ in range(500):
            while pending:
                i = pending[0]
                make, tau, steps, dtype, corr = MIX[i]
                rho0, u0, _ = alone_results[i]
                slot = pool.try_admit(rho0, u0, tau, steps, dtype=dtype, bulk_correction=corr)
                if slot is None:
                    break
                active[slot] = i
                pending.pop(0)
            pool.run(5)
            for slot in pool.poll():
                i = active.pop(slot)
                rho, u, _, _ = alone_results[i][2]
                r2, u2, _ = pool.moments(slot, raise_on_domain=False)
                assert np.array_equal(r2, rho) and np.array_equal(u2, u)
                pool.release(slot)
                checked += 1
            if not pending and not active:
                break
        assert checked == len(MIX)
        st = pool.stats()
        assert st["used_slots"] == 0 and st["free_bytes"] == st["largest_free_block"]


def test_pool_admission_limits():
    lbm = _lbm()
    rho0, u0 = workloads.taylor_green_2d(64)
    with lbm.Pool(GiB // 16, max_slots=2) as pool:
        a = pool.admit(rho0, u0, 0.6, 10)
        b = pool.admit(rho0, u0, 0.6, 10)
        with pytest.raises(lbm.LBMError) as e:
            pool.admit(rho0, u0, 0.6, 10)
        assert e.value.status == lbm.LBM_EBUSY
        pool.release(a)
        assert pool.try_admit(rho0, u0, 0.6, 10) is not None
        assert pool.slot_info(b)["steps_remaining"] == 10
    # arena budget: a slot larger than the free arena is refused with ENOMEM
    big_r, big_u = workloads.taylor_green_3d(64)
    need = lbm.lbm_pool_slot_bytes(lbm.make_config(27, (64, 64, 64), 0.6, "fp32_dev"))
    with lbm.Pool(lbm.lbm_pool_table_bytes(4) + need + (1 << 20), max_slots=4) as pool:
        s = pool.admit(big_r, big_u, 0.6, 5)
        with pytest.raises(lbm.LBMError) as e:
            pool.admit(big_r, big_u, 0.6, 5)
        assert e.value.status == lbm.LBM_ENOMEM
        pool.release(s)
        pool.admit(big_r, big_u, 0.6, 5)


def test_pool_failure_isolation():
    """A slot whose state leaves the equilibrium's domain is flagged alone."""
    lbm = _lbm()
    good_r, good_u = workloads.taylor_green_2d(32, u0=0.05)
    bad_r, bad_u = workloads.random_field((16, 16), seed=70, umax=0.99, rho_lo=0.3, rho_hi=2.0)
    _, _, bad_count = oracle.run(bad_r, bad_u, 0.5001, 6)
    assert bad_count > 0
    with lbm.Pool(GiB // 16, max_slots=4) as pool:
        g = pool.admit(good_r, good_u, 0.51, 6, dtype="fp64")
        b = pool.admit(bad_r, bad_u, 0.5001, 6, dtype="fp64")
        pool.run(6)
        assert set(pool.poll()) == {g, b}
        pool.moments(g)
        with pytest.raises(lbm.LBMDomainError):
            pool.moments(b)
        # an initial state outside the domain is refused and takes no slot
        u_bad = good_u.copy()
        u_bad[0, 3, 3] = 1.5
        with pytest.raises(lbm.LBMDomainError):
            pool.admit(good_r, u_bad, 0.6, 5)
        assert pool.stats()["used_slots"] == 2


@pytest.mark.parametrize("persistent", [0, 1])
def test_pool_matches_oracle(persistent):
    lbm = _lbm()
    cases = [(workloads.random_field((13, 21), seed=5, umax=0.3), 0.53, 9, True),
             (workloads.taylor_green_3d(10, u0=0.1), 0.6, 12, False),
             (workloads.random_field((7, 50), seed=6, umax=0.4), 0.9, 17, True)]
    with lbm.Pool(GiB // 16, max_slots=8, tuning=lbm.make_pool_tuning(persistent=persistent)) as pool:
        slots = [pool.admit(r, u, tau, steps, dtype="fp64", bulk_correction=corr) for (r, u), tau, steps, corr in cases]
        pool.run(100)
        pool.poll()
        for s, ((r0, u0), tau, steps, corr) in zip(slots, cases):
            rho, u, _ = pool.moments(s)
            r_ref, u_ref, _ = oracle.run(r0, u0, tau, steps, corr="min" if corr else "off")
            assert np.max(np.abs(rho - r_ref)) / np.max(np.abs(r_ref)) < 1e-12
            assert np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)) < 1e-12


def test_batched_workload_subset_matches_oracle_and_alone():
    """Seeded subset of the batched shear-wave workload (D2Q9, Nx, Ny in
    32..512, nu log-uniform): pool result == alone bitwise, and == oracle."""
    lbm = _lbm()
    specs = workloads.batch_domains(count=512, seed=2303)[:8]
    steps = 60
    with lbm.Pool(GiB, max_slots=16, tuning=lbm.make_pool_tuning(persistent=1)) as pool:
        slots = []
        fields = []
        for sp in specs:
            r0, u0 = workloads.shear_wave(sp["nx"], sp["ny"], sp["amp"])
            fields.append((r0, u0))
            slots.append(pool.admit(r0, u0, sp["tau"], steps, dtype="fp64"))
        pool.run(steps)
        assert set(pool.poll()) == set(slots)
        oracle.set_threads(16)
        for s, sp, (r0, u0) in zip(slots, specs, fields):
            rho, u, _ = pool.moments(s)
            ra, ua, _, _ = alone(r0, u0, sp["tau"], steps, "fp64", False)
            assert np.array_equal(rho, ra) and np.array_equal(u, ua)
            r_ref, u_ref, _ = oracle.run(r0, u0, sp["tau"], steps)
            assert np.max(np.abs(rho - r_ref)) / np.max(np.abs(r_ref)) < 1e-12
            assert np.max(np.abs(u - u_ref)) / np.max(np.abs(u_ref)) < 1e-12


def test_pool_retires_failed_slots():
    """A slot whose state leaves the equilibrium's domain is retired at the next
    poll (remaining steps dropped, reported with its flag); the others go on."""
    lbm = _lbm()
    good_r, good_u = workloads.taylor_green_2d(32, u0=0.05)
    bad_r, bad_u = workloads.random_field((16, 16), seed=70, umax=0.99, rho_lo=0.3, rho_hi=2.0)
    with lbm.Pool(GiB // 16, max_slots=4) as pool:
        g = pool.admit(good_r, good_u, 0.51, 100, dtype="fp64")
        b = pool.admit(bad_r, bad_u, 0.5001, 100000, dtype="fp64")
        pool.run(20)
        assert pool.poll() == [b]
        info = pool.slot_info(b)
        assert info["domain_error"] == 1 and info["finished"] == 1 and info["steps_remaining"] == 0
        assert info["steps_done"] == 20
        assert pool.slot_info(g)["steps_remaining"] == 80 and pool.slot_info(g)["domain_error"] == 0
        pool.run(1000)
        assert pool.poll() == [g]
        _, _, d = pool.moments(g)
        assert d["steps"] == 100 and not d["domain_error"]
        with pytest.raises(lbm.LBMDomainError):
            pool.moments(b)


@pytest.mark.parametrize("persistent", [0, 1])
def test_pool_two_steps_per_launch_equals_alone(persistent):
    """time_block = 2: D2Q9 classes that hold enough nodes (2^22 FP32, 2^20
    FP64) advance two steps per launch (ragged widths, whole-row and column
    tiles in one class, both storage types, FP32 with the correction and FP64
    with and without it);
    odd runs end with a one-step launch, small classes take one step per
    launch, and the buffer parity stays right across both forms.  With
    persistent = 1 the two-step classes take each run in one tile-ordered
    launch (odd runs end inside it) and the other classes in one grid-barrier
    launch.  Every slot is bitwise its single-domain run; the launch count
    shows which form ran."""
    lbm = _lbm()
    specs = [((33, 70), "fp32_dev", True, 0.6), ((64, 64), "fp64", False, 0.55), ((17, 130), "fp32_dev", False, 0.52),
             ((100, 45), "fp64", True, 0.7), ((5, 300), "fp32_dev", False, 0.58), ((48, 513), "fp64", False, 0.51),
             ((40, 32), "fp32_dev", True, 0.56),
             ((2048, 2048), "fp32_dev", True, 0.51), ((1024, 1024), "fp64", False, 0.51),
             ((1024, 1024), "fp64", True, 0.52)]  # large slots: every D2Q9 class but one takes two steps
    steps = 30
    fields = [workloads.random_field(shape, seed=100 + k, umax=0.1) for k, (shape, _, _, _) in enumerate(specs)]
    r3, u3 = workloads.taylor_green_3d(16, u0=0.05)
    with lbm.Pool(2 * GiB, max_slots=16, tuning=lbm.make_pool_tuning(64, 4, persistent, time_block=2)) as pool:
        slots = [pool.admit(r, u, tau, steps, dtype=dt, bulk_correction=corr)
                 for (r, u), (_, dt, corr, tau) in zip(fields, specs)]
        s3 = pool.admit(r3, u3, 0.55, steps, dtype="fp32_dev")  # D3Q27: one step per launch
        for k in (10, 6, 7, 7):
            pool.run(k)
        assert sorted(pool.poll()) == sorted(slots + [s3])
        # the three D2Q9 classes with a large slot (FP32 corrected, FP64 with and
        # without the correction): 5 + 3 two-step launches, then twice 3 two-step and
        # one one-step launch (odd runs); the small FP32 class and D3Q27: 30 each;
        # persistent: one launch per class and run
        assert pool.stats()["launches"] == (5 * 4 if persistent else 3 * (5 + 3 + 4 + 4) + 2 * 30)
        for s, (r, u), (_, dt, corr, tau) in zip(slots, fields, specs):
            ra, ua, da, fa = alone(r, u, tau, steps, dt, corr)
            rb, ub, db = pool.moments(s, raise_on_domain=False)
            assert db["steps"] == steps
            assert np.array_equal(ra, rb) and np.array_equal(ua, ub)
            assert np.array_equal(fa, pool.populations(s))
        ra, ua, _, fa = alone(r3, u3, 0.55, steps, "fp32_dev", False)
        assert np.array_equal(fa, pool.populations(s3))


def test_pool_async_admission_and_collect_equal_alone(alone_results):
    """Pipelined use: admissions without a synchronisation, run n + 1 enqueued
    before the results of run n are collected, reads of finished slots on the
    pool's second stream while later runs go on, releases that wait only for
    the slot's own work.  Every slot is bitwise its single-domain run; an
    initial state outside the domain is retired by collect."""
    import torch
    lbm = _lbm()
    dev = torch.device("cuda:0")
    with lbm.Pool(GiB // 4, max_slots=4) as pool:
        pending = list(range(len(MIX)))
        active = {}
        inflight = []
        checked = 0
        bad_slot = None
        for _ in range(2000):
            while pending:
                i = pending[0]
                make, tau, steps, dtype, corr = MIX[i]
                rho0, u0, _ = alone_results[i]
                cfg = lbm.make_config(lbm.LATTICE_OF_DIM[rho0.ndim], rho0.shape[::-1], tau, dtype, corr)
                rho_d = torch.from_numpy(rho0).to(dev)
                u_d = torch.from_numpy(u0).to(dev)
                try:
                    slot = lbm.lbm_pool_admit_async(pool.handle, cfg, rho_d.data_ptr(), u_d.data_ptr(), steps)
                except lbm.LBMError as e:
                    assert e.status in (lbm.LBM_EBUSY, lbm.LBM_ENOMEM)
                    break
                pool.shapes[slot] = rho0.shape
                active[slot] = i
                pending.pop(0)
            if bad_slot is None and not pending and len(active) < 4:
                # an initial state with |u_x| >= 1 at one node
                r_bad, u_bad = workloads.taylor_green_2d(32, u0=0.05)
                u_bad[0, 5, 7] = 1.25
                cfg = lbm.make_config(9, (32, 32), 0.6, "fp32_dev")
                rb, ub = torch.from_numpy(r_bad).to(dev), torch.from_numpy(u_bad).to(dev)
                bad_slot = lbm.lbm_pool_admit_async(pool.handle, cfg, rb.data_ptr(), ub.data_ptr(), 50)
                pool.shapes[bad_slot] = r_bad.shape
            pool.run(3)
            inflight.append(pool.stats()["runs"])
            if len(inflight) < 2 and (pending or active):
                continue
            for slot in lbm.lbm_pool_collect(pool.handle, inflight.pop(0)):
                if slot == bad_slot:
                    assert pool.slot_info(slot)["domain_error"] == 1
                    with pytest.raises(lbm.LBMDomainError):
                        pool.moments(slot)
                    pool.release(slot)
                    bad_slot = -1
                    continue
                i = active.pop(slot)
                rho, u, _, f = alone_results[i][2]
                r2, u2, _ = pool.moments(slot, raise_on_domain=False)
                assert np.array_equal(r2, rho) and np.array_equal(u2, u)
                assert np.array_equal(pool.populations(slot), f)
                pool.release(slot)
                checked += 1
            if not pending and not active and bad_slot == -1:
                break
        assert checked == len(MIX) and bad_slot == -1
        st = pool.stats()
        assert st["used_slots"] == 0 and st["free_bytes"] == st["largest_free_block"]


def test_persistent_barrier_timeout_retires_slots_and_pool_recovers():
    """The timeout path of the persistent form's bounded grid barrier, forced
    from the host: with a bound of 2 polls the workgroups of a full grid do not
    all arrive in time, and every one of them leaves through the bounded wait.
    poll reports LBM_EDEVICE; the slots that run advanced are retired with
    device_error and refuse reads; the next poll lists them; the barrier state
    is reset, so a later persistent run completes normally."""
    lbm = _lbm()
    fields = [workloads.shear_wave(256, 256, 0.05) for _ in range(8)]
    with lbm.Pool(GiB, max_slots=16, tuning=lbm.make_pool_tuning(persistent=1, spin_log2=1)) as pool:
        slots = [pool.admit(r, u, 0.6, 200, dtype="fp32_dev") for r, u in fields]
        pool.run(200)
        with pytest.raises(lbm.LBMError) as e:
            pool.poll()
        assert e.value.status == lbm.LBM_EDEVICE
        for s in slots:
            info = pool.slot_info(s)
            assert info["device_error"] == 1 and info["finished"] == 1 and info["domain_error"] == 0
            with pytest.raises(lbm.LBMError) as e2:
                pool.moments(s, fields=False)
            assert e2.value.status == lbm.LBM_EDEVICE
        assert sorted(pool.poll()) == sorted(slots)
        for s in slots:
            pool.release(s)
        # one-step runs need no barrier; after the reset, poll reports no error
        r, u = fields[0]
        s = pool.admit(r, u, 0.6, 1, dtype="fp32_dev")
        pool.run(1)
        assert pool.poll() == [s]
        rho, vel, _ = pool.moments(s)
        ra, ua, _, _ = alone(r, u, 0.6, 1, "fp32_dev", False)
        assert np.array_equal(rho, ra) and np.array_equal(vel, ua)


def test_tile_ordered_timeout_retires_slots_and_pool_recovers():
    """The timeout path of the tile-ordered persistent form, forced from the
    host: four 1024^2 FP32 slots take 256 column tiles, one per workgroup, and
    with a bound of 2 polls a tile's second iteration does not find all eight
    neighbours done in time; the workgroup reports the timeout and every other
    one leaves at its next wait.  poll reports LBM_EDEVICE, the slots are
    retired with device_error, and a later run (one step, which waits for no
    neighbour) completes and equals the single-domain run."""
    lbm = _lbm()
    fields = [workloads.shear_wave(1024, 1024, 0.05) for _ in range(4)]
    tuning = lbm.make_pool_tuning(64, 4, persistent=1, time_block=2, spin_log2=1)
    with lbm.Pool(GiB, max_slots=8, tuning=tuning) as pool:
        slots = [pool.admit(r, u, 0.6, 40, dtype="fp32_dev") for r, u in fields]
        pool.run(40)
        assert pool.stats()["launches"] == 1
        with pytest.raises(lbm.LBMError) as e:
            pool.poll()
        assert e.value.status == lbm.LBM_EDEVICE
        for s in slots:
            info = pool.slot_info(s)
            assert info["device_error"] == 1 and info["finished"] == 1 and info["domain_error"] == 0
            with pytest.raises(lbm.LBMError) as e2:
                pool.moments(s, fields=False)
            assert e2.value.status == lbm.LBM_EDEVICE
        assert sorted(pool.poll()) == sorted(slots)
        for s in slots:
            pool.release(s)
        r, u = fields[0]
        s = pool.admit(r, u, 0.6, 1, dtype="fp32_dev")
        pool.run(1)
        assert pool.poll() == [s]
        rho, vel, _ = pool.moments(s)
        ra, ua, _, _ = alone(r, u, 0.6, 1, "fp32_dev", False)
        assert np.array_equal(rho, ra) and np.array_equal(vel, ua)


@pytest.mark.parametrize("form", ["rows", "fit", "flat", "persistent", "persistent-flat", "two-step",
                                  "two-step-persistent"])
def test_pool_kernels_store_only_inside_their_slots(form):
    """Every store of the pool kernels, padding lanes included, stays inside its
    slot's own buffers: canary bytes written into the arena around the slots
    (a released block between two slots, the free region after them, the
    unused words beside the grid-barrier counter and error word, and the
    tables of classes that do not run) are intact after runs of each launch
    form, and the slots equal their single-domain runs."""
    import torch
    lbm = _lbm()
    tun = {"rows": dict(tile_x=64, tile_y=4), "fit": dict(tile_x=64, tile_y=4, row_fit=1),
           "flat": dict(tile_x=64, tile_y=4, flat=1), "persistent": dict(persistent=1),
           "persistent-flat": dict(persistent=1, flat=1),
           "two-step": dict(tile_x=64, tile_y=4, time_block=2),
           "two-step-persistent": dict(tile_x=64, tile_y=4, time_block=2, persistent=1)}[form]
    tuning = lbm.make_pool_tuning(**tun)
    # ragged widths (padding lanes), a D3Q27 cube, and D2Q9 slots large enough for two-step launches
    specs = [((33, 70), "fp32_dev"), ((17, 130), "fp32_dev"), ((9, 11, 13), "fp32_dev"), ((2100, 2048), "fp32_dev"),
             ((37, 100), "fp64"), ((1100, 1030), "fp64")]
    fields = [workloads.random_field(shape, seed=300 + k, umax=0.1) for k, (shape, _) in enumerate(specs)]
    max_slots = 8
    tb = lbm.lbm_pool_table_bytes(max_slots)
    sizes = [lbm.lbm_pool_slot_bytes(lbm.make_config(lbm.LATTICE_OF_DIM[len(sh)], sh[::-1], 0.6, dt), tuning)
             for sh, dt in specs]
    arena = tb + (2 << 20) + sum(sizes) + (8 << 20)
    steps = 12
    with lbm.Pool(arena, max_slots=max_slots, tuning=tuning) as pool:
        base = (pool._arena.data_ptr() + 255) // 256 * 256 - pool._arena.data_ptr()
        buf = pool._arena
        r_sp, u_sp = workloads.taylor_green_2d(16)
        slots, offs = [], []
        off = tb
        gaps = []
        for k, ((r, u), (sh, dt)) in enumerate(zip(fields, specs)):
            if k == 3:
                # a small slot between two others, released below: its block becomes a gap
                sp = pool.admit(r_sp, u_sp, 0.6, 1)
                sp_bytes = pool.slot_info(sp)["bytes"]
                gaps.append((off, sp_bytes))
                off += sp_bytes
                spacer_slot = sp
            slots.append(pool.admit(r, u, 0.6, steps, dtype=dt))
            assert pool.slot_info(slots[-1])["bytes"] == sizes[k]
            offs.append(off)
            off += sizes[k]
        pool.release(spacer_slot)
        gaps.append((off, min(8 << 20, arena - off)))  # free region after the last slot
        torch.cuda.synchronize()
        CAN = 0xA5
        # canaries: the gaps, the words between the barrier counter and the error word and
        # after it (the table region's 512-byte barrier block), and the unused class tables;
        # the table region is 16 class tables, the 512-byte barrier block, the gather area
        regions = list(gaps)
        n_classes = 16
        gather_bytes = ((8 * max_slots + 255) // 256 * 256) + ((4 * max_slots + 255) // 256 * 256)
        class_bytes = (tb - 512 - gather_bytes) // n_classes
        barrier_off = n_classes * class_bytes
        regions += [(barrier_off + 4, 252), (barrier_off + 260, 252)]
        used_classes = {(8 if len(sh) == 3 else 0) + 2 * (0 if dt == "fp64" else 1) for sh, dt in specs}
        regions += [(c * class_bytes, class_bytes) for c in range(n_classes) if c not in used_classes]
        for o, ln in regions:
            buf[base + o: base + o + ln].fill_(CAN)
        torch.cuda.synchronize()
        for k in (6, 6):  # even runs: the two-step form takes both D2Q9 classes
            pool.run(k)
        assert sorted(pool.poll()) == sorted(slots)
        if form == "two-step":
            assert pool.stats()["launches"] == (3 + 3) * 2 + 12  # two D2Q9 classes two-step, D3Q27 one-step
        if form == "two-step-persistent":
            assert pool.stats()["launches"] == 3 * 2  # one launch per class and run
        for o, ln in regions:
            seg = buf[base + o: base + o + ln]
            assert bool(torch.all(seg == CAN)), (form, o, ln)
        for s, (r, u), (sh, dt) in zip(slots, fields, specs):
            ra, ua, _, _ = alone(r, u, 0.6, steps, dt, False)
            rb, ub, _ = pool.moments(s)
            assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (form, sh, dt)


@pytest.mark.parametrize("form", ["launches", "tile_ordered", "tile_ordered_5wg"])
@pytest.mark.parametrize("dtype", ["fp32_dev", "fp64"])
def test_pool_two_step_mixed_step_counts_equal_alone(dtype, form):
    """Two steps per launch when the slots of a class take different numbers of
    steps in one run: launch L covers, in two-step tiles, the slots with at
    least 2 L + 2 steps and then, in a one-step launch, those whose last step
    is 2 L + 1, whole-row and column-tile slots alike.  The tile-ordered
    persistent form takes each run in one launch: a slot with s steps takes
    ceil(s / 2) iterations, the last of one step when s is odd; with 5
    workgroups each owns many tiles of several slots with different iteration
    counts.  Each slot equals its single-domain run bitwise after every run."""
    lbm = _lbm()
    extra = {"launches": {}, "tile_ordered": dict(persistent=1), "tile_ordered_5wg": dict(persistent=1, workgroups=5)}
    tuning = lbm.make_pool_tuning(64, 4, time_block=2, time_rows=8, **extra[form])
    big = (2048, 2100) if dtype == "fp32_dev" else (1030, 1100)
    specs = [(big, 13), ((40, 70), 10), ((33, 100), 7), ((64, 512), 4), ((20, 700), 11), ((17, 129), 1),
             ((90, 64), 12)]
    fields = [workloads.random_field(shape, seed=400 + k, umax=0.1) for k, (shape, _) in enumerate(specs)]
    with lbm.Pool(2 * GiB, max_slots=16, tuning=tuning) as pool:
        slots = [pool.admit(r, u, 0.55, steps, dtype=dtype) for (r, u), (_, steps) in zip(fields, specs)]
        done = set()
        for k in (5, 100):  # the first run cuts every budget at 5 steps (odd), the second finishes them
            launches = pool.stats()["launches"]
            pool.run(k)
            if form != "launches":
                assert pool.stats()["launches"] == launches + 1
            done |= set(pool.poll())
            for s, (r, u), (_, steps) in zip(slots, fields, specs):
                n = min(steps, 5 if k == 5 else steps)
                ra, ua, _, _ = alone(r, u, 0.55, n, dtype, False)
                rb, ub, db = pool.moments(s)
                assert db["steps"] == n
                assert np.array_equal(ra, rb) and np.array_equal(ua, ub), (s, n)
        assert done == set(slots)
