"""z-slabs with halo exchange (lbm_config.z_halo, lbm_halo_pack/unpack): a
periodic D3Q27 domain split along z into slabs that exchange the populations
crossing their faces after every step advances bitwise as the whole domain
(streaming of the LBGK equation, Sec. "Basic concepts": only populations with
c_z = +1 cross a face upwards, c_z = -1 downwards).  Slabs here live on one
GPU and exchange through device buffers, which is what a send/recv between
GPUs would carry."""
import numpy as np
import pytest

import oracle
from paper_2303_08163_amd import workloads

pytestmark = pytest.mark.gpu


def _lbm():
    from paper_2303_08163_amd import lbm
    return lbm


def ring_run(rho0, u0, splits, tau, steps, dtype, corr, eq="entropic", tuning=None, split_faces=False):
    """Advance slabs of the given plane counts (a ring, periodic in z) and return
    (rho, u, populations) gathered along z, and the slabs' diagnostics."""
    import torch
    lbm = _lbm()
    assert sum(splits) == rho0.shape[0]
    bounds = np.cumsum([0] + list(splits))
    slabs = [lbm.Domain(rho0[a:b], u0[:, a:b], tau, dtype=dtype, bulk_correction=corr, equilibrium=eq,
                        tuning=tuning, z_halo=True) for a, b in zip(bounds[:-1], bounds[1:])]
    S = len(slabs)
    nb = slabs[0].halo_bytes()
    assert nb == 9 * rho0.shape[1] * rho0.shape[2] * (8 if dtype == "fp64" else 4)
    lo = [torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(S)]
    hi = [torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(S)]

    def exchange():
        for k, s in enumerate(slabs):
            if split_faces:  # one face per call
                s.halo_pack(lo[k], None)
                s.halo_pack(None, hi[k])
            else:
                s.halo_pack(lo[k], hi[k])
        for k, s in enumerate(slabs):
            if split_faces:
                s.halo_unpack(hi[(k - 1) % S], None)
                s.halo_unpack(None, lo[(k + 1) % S])
            else:
                s.halo_unpack(hi[(k - 1) % S], lo[(k + 1) % S])

    try:
        exchange()
        for _ in range(steps):
            for s in slabs:
                s.step(1)
            exchange()
        out = [s.moments(raise_on_domain=False) for s in slabs]
        pops = [s.populations().reshape(27, -1, rho0.shape[1], rho0.shape[2]) for s in slabs]
    finally:
        for s in slabs:
            s.close()
    rho = np.concatenate([o[0] for o in out], axis=0)
    u = np.concatenate([o[1] for o in out], axis=1)
    return rho, u, np.concatenate(pops, axis=1), [o[2] for o in out]


def whole_run(rho0, u0, tau, steps, dtype, corr, eq="entropic", tuning=None):
    lbm = _lbm()
    with lbm.Domain(rho0, u0, tau, dtype=dtype, bulk_correction=corr, equilibrium=eq, tuning=tuning) as d:
        d.step(steps)
        rho, u, diag = d.moments(raise_on_domain=False)
        f = d.populations().reshape(27, *rho0.shape)
    return rho, u, f, diag


CASES = [  # (grid (nz, ny, nx), splits, tau, steps, dtype, corr)
    ((8, 13, 19), [5, 3], 0.56, 7, "fp64", False),
    ((8, 13, 19), [5, 3], 0.56, 7, "fp32_dev", True),
    ((7, 10, 24), [7], 0.6, 6, "fp64", True),
    ((8, 9, 20), [1, 2, 3, 2], 0.53, 5, "fp32_dev", False),
    ((6, 4, 256), [2, 4], 0.51, 5, "fp32_dev", False),   # vector kernel, one wavefront per row
    ((6, 3, 128), [3, 3], 0.58, 4, "fp64", True),        # vector kernel, FP64 pairs
    ((5, 3, 512), [2, 3], 0.52, 3, "fp32_dev", True),    # vector kernel across wavefronts
    ((3, 1, 1), [1, 1, 1], 0.6, 4, "fp64", False),       # 1 x 1 cross-section, one-plane slabs
    ((4, 2, 5), [2, 2], 0.55, 5, "fp32_dev", True),      # rows narrower than the 16-element pitch
    ((4, 3, 300), [3, 1], 0.57, 4, "fp64", True),        # packed runs longer than a workgroup
]


@pytest.mark.parametrize("grid,splits,tau,steps,dtype,corr", CASES)
def test_slab_ring_equals_whole_domain_bitwise(grid, splits, tau, steps, dtype, corr):
    rho0, u0 = workloads.random_field(grid, seed=91, umax=0.15)
    r1, u1, f1, diags = ring_run(rho0, u0, splits, tau, steps, dtype, corr)
    r2, u2, f2, diag = whole_run(rho0, u0, tau, steps, dtype, corr)
    print(f"[slab] {grid} splits {splits} {dtype} corr={corr}: max |drho| {np.max(np.abs(r1 - r2)):.3e}", flush=True)
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2) and np.array_equal(f1, f2)
    assert all(d["steps"] == steps and not d["domain_error"] for d in diags)
    assert abs(sum(d["mass"] for d in diags) - diag["mass"]) < 1e-9 * diag["mass"]


@pytest.mark.parametrize("eq", ["poly2", "product"])
def test_slab_ring_polynomial_equilibria(eq):
    rho0, u0 = workloads.random_field((6, 7, 33), seed=92, umax=0.12)
    r1, u1, f1, _ = ring_run(rho0, u0, [4, 2], 0.55, 5, "fp64", True, eq=eq, split_faces=(eq == "product"))
    r2, u2, f2, _ = whole_run(rho0, u0, 0.55, 5, "fp64", True, eq=eq)
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2) and np.array_equal(f1, f2)


def test_slab_ring_scalar_tuning_equals_vector():
    """A ring of slabs run with one node per thread equals the default vector kernels."""
    lbm = _lbm()
    rho0, u0 = workloads.random_field((4, 4, 256), seed=93, umax=0.1)
    a = ring_run(rho0, u0, [1, 3], 0.52, 4, "fp32_dev", False, tuning=lbm.make_tuning(64, 4, -1, 1, 0))
    b = ring_run(rho0, u0, [1, 3], 0.52, 4, "fp32_dev", False)
    assert np.array_equal(a[0], b[0]) and np.array_equal(a[2], b[2])


def test_slab_ring_matches_oracle():
    """The gathered slabs against the FP64 oracle of the whole periodic domain."""
    rho0, u0 = workloads.random_field((9, 11, 17), seed=94, umax=0.15)
    r1, u1, _, _ = ring_run(rho0, u0, [4, 5], 0.57, 10, "fp64", True)
    r_ref, u_ref, bad = oracle.run(rho0, u0, 0.57, 10, corr="min")
    assert bad == 0
    assert np.max(np.abs(r1 - r_ref)) / np.max(np.abs(r_ref)) < 1e-12
    assert np.max(np.abs(u1 - u_ref)) / np.max(np.abs(u_ref)) < 1e-12


def test_slab_errors():
    import torch
    lbm = _lbm()
    rho0, u0 = workloads.random_field((4, 5, 6), seed=95, umax=0.1)
    buf = torch.empty(9 * 5 * 6 * 8, dtype=torch.uint8, device="cuda:0")
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64", z_halo=True) as s:
        with pytest.raises(lbm.LBMError):
            s.step(2)  # a slab needs an exchange between steps
        with pytest.raises(lbm.LBMError):
            s.halo_pack(None, None)
        with pytest.raises(lbm.LBMError):
            s.halo_unpack(None, None)
        s.step(0)
        s.step(1)
        assert s.moments(raise_on_domain=False)[2]["steps"] == 1
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64") as d:
        assert d.halo_bytes() == 0
        with pytest.raises(lbm.LBMError):
            d.halo_pack(buf, buf)
        d.step(3)  # periodic domains take any step count


def _moments_ring(rho0, u0, splits, tau, steps, dtype):
    """Moments only (full-size grids): rings of slabs as in ring_run."""
    import torch
    lbm = _lbm()
    bounds = np.cumsum([0] + list(splits))
    slabs = [lbm.Domain(rho0[a:b], u0[:, a:b], tau, dtype=dtype, z_halo=True)
             for a, b in zip(bounds[:-1], bounds[1:])]
    S = len(slabs)
    nb = slabs[0].halo_bytes()
    lo = [torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(S)]
    hi = [torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(S)]

    def exchange():
        for k, s in enumerate(slabs):
            s.halo_pack(lo[k], hi[k])
        for k, s in enumerate(slabs):
            s.halo_unpack(hi[(k - 1) % S], lo[(k + 1) % S])

    try:
        exchange()
        for _ in range(steps):
            for s in slabs:
                s.step(1)
            exchange()
        out = [s.moments(raise_on_domain=False) for s in slabs]
    finally:
        for s in slabs:
            s.close()
    return np.concatenate([o[0] for o in out], axis=0), np.concatenate([o[1] for o in out], axis=1)


@pytest.mark.parametrize("planes,splits", [(32, [32]), (64, [32, 32])])
def test_slab_full_size_bench_shape(planes, splits):
    """The benchmark's slab (256 x 256 x 32, FP32, default launch shape, planes
    of the 256^3 Taylor-Green field): as its own neighbour it advances as the
    periodic 256 x 256 x 32 domain, and two such slabs as the 256 x 256 x 64
    domain, bitwise."""
    lbm = _lbm()
    rho0, u0 = workloads.taylor_green_3d(256, u0=0.05, planes=(0, planes))
    r1, u1 = _moments_ring(rho0, u0, splits, 0.5005, 4, "fp32_dev")
    with lbm.Domain(rho0, u0, 0.5005, dtype="fp32_dev") as d:
        d.step(4)
        r2, u2, _ = d.moments()
    print(f"[slab full size] 256x256x{planes} splits {splits}: max |du| {np.max(np.abs(u1 - u2)):.3e}", flush=True)
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2)


def fused_ring_run(rho0, u0, splits, tau, steps, dtype, corr, eq="entropic", tuning=None):
    """Rings of slabs advanced by lbm_step_halo: the entering populations are
    read from the neighbours' send buffers of the previous step (two sets,
    alternating with the step's parity), seeded by lbm_halo_pack."""
    import torch
    lbm = _lbm()
    bounds = np.cumsum([0] + list(splits))
    slabs = [lbm.Domain(rho0[a:b], u0[:, a:b], tau, dtype=dtype, bulk_correction=corr, equilibrium=eq,
                        tuning=tuning, z_halo=True) for a, b in zip(bounds[:-1], bounds[1:])]
    S = len(slabs)
    nb = slabs[0].halo_bytes()
    buf = [[[torch.empty(nb, dtype=torch.uint8, device="cuda:0") for _ in range(2)] for _ in range(2)]
           for _ in range(S)]  # buf[slab][parity][face]
    try:
        for k, s in enumerate(slabs):
            s.halo_pack(buf[k][1][0], buf[k][1][1])
        for t in range(steps):
            p = t % 2
            for k, s in enumerate(slabs):
                s.step_halo(buf[(k - 1) % S][1 - p][1], buf[(k + 1) % S][1 - p][0], buf[k][p][0], buf[k][p][1])
        out = [s.moments(raise_on_domain=False) for s in slabs]
        pops = [s.populations().reshape(27, -1, rho0.shape[1], rho0.shape[2]) for s in slabs]
        # the last step's send buffers hold what lbm_halo_pack now writes
        p = (steps - 1) % 2
        for k, s in enumerate(slabs):
            lo = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
            hi = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
            s.halo_pack(lo, hi)
            assert torch.equal(lo, buf[k][p][0]) and torch.equal(hi, buf[k][p][1])
    finally:
        for s in slabs:
            s.close()
    rho = np.concatenate([o[0] for o in out], axis=0)
    u = np.concatenate([o[1] for o in out], axis=1)
    return rho, u, np.concatenate(pops, axis=1)


FUSED_CASES = [  # (grid (nz, ny, nx), splits, tau, steps, dtype, corr, eq)
    ((8, 13, 19), [5, 3], 0.56, 7, "fp64", True, "entropic"),      # one node per thread, ragged rows
    ((8, 9, 20), [1, 2, 3, 2], 0.53, 5, "fp32_dev", False, "entropic"),
    ((7, 10, 24), [7], 0.6, 6, "fp32_dev", True, "poly2"),
    ((6, 4, 256), [2, 4], 0.51, 5, "fp32_dev", False, "entropic"),  # vector kernel, one wavefront per row
    ((6, 3, 128), [3, 3], 0.58, 4, "fp64", True, "product"),       # vector kernel, FP64 pairs
    ((5, 3, 512), [2, 3], 0.52, 3, "fp32_dev", True, "entropic"),   # vector kernel across wavefronts
    ((3, 1, 1), [1, 1, 1], 0.6, 4, "fp64", False, "entropic"),      # 1 x 1 cross-section
    ((4, 3, 300), [3, 1], 0.57, 4, "fp32_dev", True, "product"),    # ragged rows over several tiles
]


@pytest.mark.parametrize("grid,splits,tau,steps,dtype,corr,eq", FUSED_CASES)
def test_fused_halo_steps_equal_whole_domain_bitwise(grid, splits, tau, steps, dtype, corr, eq):
    rho0, u0 = workloads.random_field(grid, seed=97, umax=0.15)
    r1, u1, f1 = fused_ring_run(rho0, u0, splits, tau, steps, dtype, corr, eq)
    r2, u2, f2, _ = whole_run(rho0, u0, tau, steps, dtype, corr, eq)
    print(f"[slab fused] {grid} splits {splits} {dtype} {eq} corr={corr}", flush=True)
    assert np.array_equal(r1, r2) and np.array_equal(u1, u2) and np.array_equal(f1, f2)


def test_fused_and_plane_steps_mix():
    """Steps through the halo planes (pack, unpack, lbm_step) and fused steps
    can alternate on the same slabs: each leaves the state the other expects."""
    import torch
    lbm = _lbm()
    rho0, u0 = workloads.random_field((6, 5, 16), seed=98, umax=0.12)
    a = lbm.Domain(rho0[:3], u0[:, :3], 0.57, dtype="fp64", z_halo=True)
    b = lbm.Domain(rho0[3:], u0[:, 3:], 0.57, dtype="fp64", z_halo=True)
    nb = a.halo_bytes()
    t = {key: torch.empty(nb, dtype=torch.uint8, device="cuda:0") for key in
         ("alo", "ahi", "blo", "bhi", "alo2", "ahi2", "blo2", "bhi2")}
    try:
        for step in range(6):
            a.halo_pack(t["alo"], t["ahi"])
            b.halo_pack(t["blo"], t["bhi"])
            if step % 2 == 0:  # plane form
                a.halo_unpack(t["bhi"], t["blo"])
                b.halo_unpack(t["ahi"], t["alo"])
                a.step(1)
                b.step(1)
            else:  # fused form
                a.step_halo(t["bhi"], t["blo"], t["alo2"], t["ahi2"])
                b.step_halo(t["ahi"], t["alo"], t["blo2"], t["bhi2"])
        rho = np.concatenate([a.moments()[0], b.moments()[0]], axis=0)
    finally:
        a.close()
        b.close()
    r2, _, _, _ = whole_run(rho0, u0, 0.57, 6, "fp64", False)
    assert np.array_equal(rho, r2)


def test_fused_halo_errors():
    import torch
    lbm = _lbm()
    rho0, u0 = workloads.random_field((4, 5, 6), seed=99, umax=0.1)
    b = [torch.empty(9 * 5 * 6 * 8, dtype=torch.uint8, device="cuda:0") for _ in range(4)]
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64", z_halo=True) as s:
        with pytest.raises(lbm.LBMError):
            s.step_halo(b[0], b[1], b[0], b[2])  # receive buffer reused as a send buffer
        with pytest.raises(lbm.LBMError):
            s.step_halo(b[0], b[1], b[2], b[2])  # the same send buffer twice
        with pytest.raises(lbm.LBMError):
            lbm.lbm_step_halo(s.handle, b[0].data_ptr(), None, b[2].data_ptr(), b[3].data_ptr())
        s.halo_pack(b[0], b[1])
        s.step_halo(b[1], b[0], b[2], b[3])  # its own neighbour
        assert s.moments(raise_on_domain=False)[2]["steps"] == 1
    with lbm.Domain(rho0, u0, 0.6, dtype="fp64") as d:
        with pytest.raises(lbm.LBMError):
            d.step_halo(b[0], b[1], b[2], b[3])
