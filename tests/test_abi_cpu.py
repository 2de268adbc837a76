"""CPU checks of the C-ABI library: it loads, exports every function the
header declares, and its host-only logic (configuration validation, workspace
sizing, status strings, argument checks that precede any GPU call) behaves as
documented.  No kernel is launched here."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


@pytest.fixture(scope="module")
def lbm():
    from paper_2303_08163_amd import lbm as m
    if not os.path.exists(m.LIB_PATH):
        from paper_2303_08163_amd import build
        build.build()
    m.load_library()
    return m


def declared_functions():
    names = set()
    for fn in os.listdir(os.path.join(ROOT, "include")):
        if fn.endswith(".h"):
            text = open(os.path.join(ROOT, "include", fn)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(lbm_[a-z_0-9]+)\s*\(", text))
    return sorted(names)


def test_every_declared_symbol_is_exported(lbm):
    lib = lbm.load_library()
    names = declared_functions()
    assert "lbm_step" in names and "lbm_create" in names
    for name in names:
        assert hasattr(lib, name), name
    assert set(lbm.EXPORTS) == set(names)


def test_status_strings(lbm):
    for code in (0, -1, -2, -3, -4, -5):
        assert lbm.lbm_status_string(code).startswith("LBM_")
    assert lbm.lbm_status_string(7) == "unknown status"
    assert "gfx950" in lbm.lbm_version()


def _cfg(lbm, **kw):
    base = dict(lattice=9, shape=(64, 32), tau=0.6, dtype="fp64", bulk_correction=False, rho0=1.0,
                equilibrium="entropic")
    base.update(kw)
    return lbm.make_config(base["lattice"], base["shape"], base["tau"], base["dtype"], base["bulk_correction"],
                           base["rho0"], base["equilibrium"])


def test_workspace_bytes_layout(lbm):
    # D2Q9 FP64 64x32: two buffers of 9 * 2048 doubles, flag, diag, partials
    n = 64 * 32
    buf = 9 * n * 8
    red = min(1024, (n + 255) // 256)
    expect = 2 * buf + 256 + 256 + ((red * 7 * 8 + 255) // 256) * 256
    assert lbm.lbm_workspace_bytes(_cfg(lbm)) == expect
    # FP32 deviation storage halves the buffers
    assert lbm.lbm_workspace_bytes(_cfg(lbm, dtype="fp32_dev")) == expect - buf
    # D3Q27 256^3 FP32: 2 x 27 x 256^3 x 4 bytes plus scratch
    b3 = lbm.lbm_workspace_bytes(_cfg(lbm, lattice=27, shape=(256, 256, 256), dtype="fp32_dev"))
    assert 2 * 27 * 256 ** 3 * 4 < b3 < 2 * 27 * 256 ** 3 * 4 + 2 ** 20
    # plane layout: padding adds whole 64-element blocks per plane
    t = lbm.make_tuning(0, 0, 100, layout=lbm.LBM_LAYOUT_PLANES)
    assert lbm.lbm_workspace_bytes(_cfg(lbm), t) == expect + 2 * 9 * 128 * 8
    # row-interleaved layout (default): each population run padded to 16 elements
    e70 = lbm.lbm_workspace_bytes(_cfg(lbm, shape=(70, 32)))
    assert e70 == 2 * 9 * 80 * 32 * 8 + 256 + 256 + ((9 * 7 * 8 + 255) // 256) * 256
    # D1Q3: one row of 3 runs; 64 x 3 doubles per buffer, one reduction block
    assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(64,))) == 2 * 3 * 64 * 8 + 256 + 256 + 256
    assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(70,))) == 2 * ((3 * 80 * 8 + 255) // 256) * 256 + 768
    # below 16 the run is not padded
    assert lbm.lbm_workspace_bytes(_cfg(lbm, shape=(5, 3))) == 2 * 1280 + 256 + 256 + 256  # 1080 B buffers, 256-aligned


@pytest.mark.parametrize("bad", [
    dict(tau=0.5), dict(tau=0.3), dict(tau=float("nan")), dict(tau=float("inf")),
    dict(lattice=19), dict(dtype=7), dict(shape=(0, 5)), dict(shape=(5, 0)),
    dict(shape=(4, 4, 2)), dict(lattice=27, shape=(4, 4, 0)), dict(dtype="fp32_dev", rho0=0.0),
    dict(dtype="fp32_dev", rho0=-1.0), dict(shape=(70000, 70000)), dict(lattice=27, shape=(2, 2, 2 ** 30)), dict(shape=(2 ** 31, 1)),
    dict(lattice=3, shape=(64, 2)), dict(lattice=3, shape=(64, 1, 2)), dict(lattice=3, shape=(0,)),
    dict(equilibrium=3), dict(equilibrium=-1), dict(equilibrium="poly2", dtype="fp32_dev_mixed"),
    dict(equilibrium="product", dtype="fp32_dev_f32"),
])
def test_invalid_configs_are_rejected(lbm, bad):
    assert lbm.lbm_workspace_bytes(_cfg(lbm, **bad)) == 0


@pytest.mark.parametrize("tun", [(48, 4, 0), (64, 8, 0), (3, 64, 0), (64, 5, 0), (64, 4, 1 << 21, 1, 0, 2),
                                 (64, 4, 0, 3), (64, 4, 0, 4), (64, 4, 0, 2, 2), (64, 4, 0, 2, 4), (64, 4, 0, 1, 1),
                                 (32, 8, 0, 2, 1), (0, 0, -1, 0, -1, 3)])
def test_invalid_tuning_rejected(lbm, tun):
    # cfg: D2Q9 FP64 64 x 32 (4 nodes per thread needs FP32; 64 * 2 does not divide 64)
    assert lbm.lbm_workspace_bytes(_cfg(lbm), lbm.make_tuning(*tun)) == 0


def test_valid_tunings_accepted(lbm):
    cfg = _cfg(lbm, shape=(256, 8), dtype="fp32_dev")
    for tun in [(0, 0, -1, 0, -1, 0), (64, 4, 0, 4, 3, 1), (64, 1, 0, 2, 1, 2), (128, 2, 64, 2, 0, 2),
                (256, 1, 0, 1, 0, 1), (32, 8, 0, 1, 0, 0)]:
        assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(*tun)) > 0, tun


def test_time_block_configs(lbm):
    """Two steps per launch: D2Q9, FP64 or FP32_DEV, rows layout, nx >= 64;
    the workspace is that of the one-step domain."""
    two = lbm.make_tuning(time_block=2)
    for dt in ("fp64", "fp32_dev"):
        for nx in (64, 192, 4096):
            cfg = _cfg(lbm, shape=(nx, 5), dtype=dt)
            assert lbm.lbm_workspace_bytes(cfg, two) == lbm.lbm_workspace_bytes(cfg) > 0
            assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_block=2, time_rows=5)) > 0
            assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_block=2, time_rows=6)) == 0
            assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_block=2, time_rows=-1)) == 0
    for nx in (65, 96, 100, 1000):  # ragged widths: the last tile of a row is partial
        for dt in ("fp64", "fp32_dev"):
            assert lbm.lbm_workspace_bytes(_cfg(lbm, shape=(nx, 8), dtype=dt), two) > 0
    refused = [_cfg(lbm, shape=(63, 8)), _cfg(lbm, shape=(40, 8), dtype="fp32_dev"),
               _cfg(lbm, lattice=27, shape=(64, 8, 8)), _cfg(lbm, lattice=3, shape=(15,)),
               _cfg(lbm, shape=(64, 8), dtype="fp32_dev_mixed")]
    for cfg in refused:
        assert lbm.lbm_workspace_bytes(cfg, two) == 0
    assert b"time_block" in lbm.load_library().lbm_last_error()
    cfg = _cfg(lbm, shape=(64, 8))
    assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(layout=lbm.LBM_LAYOUT_PLANES, time_block=2)) == 0
    assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_block=3)) == 0
    assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_rows=4)) == 0  # rows without two steps
    assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(time_block=1)) > 0


def test_d1q3_time_block_configs(lbm):
    """K = 2, 4 or 8 steps per launch on D1Q3: FP64 or FP32_DEV, nx >= 16;
    D2Q9 takes 2 only."""
    for K in (2, 4, 8):
        for nx in (16, 64, 1031, 1032, 5000):
            for dt in ("fp32_dev", "fp64"):
                assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(nx,), dtype=dt),
                                               lbm.make_tuning(time_block=K)) > 0, (K, nx, dt)
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(15,), dtype="fp32_dev"),
                                       lbm.make_tuning(time_block=K)) == 0
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(15,)), lbm.make_tuning(time_block=K)) == 0
    for K in (3, 5, 16):
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(4096,)), lbm.make_tuning(time_block=K)) == 0
    for K in (4, 8):
        assert lbm.lbm_workspace_bytes(_cfg(lbm, shape=(4096, 64)), lbm.make_tuning(time_block=K)) == 0
    for eq in ("poly2", "product"):  # every equilibrium, on both lattices
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(4096,), equilibrium=eq),
                                       lbm.make_tuning(time_block=4)) > 0
        assert lbm.lbm_workspace_bytes(_cfg(lbm, shape=(128, 8), equilibrium=eq), lbm.make_tuning(time_block=2)) > 0
    assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(4096,)), lbm.make_tuning(time_block=4, time_rows=2)) == 0


def test_polynomial_equilibria_configs(lbm):
    """The polynomial kinds take both production storage modes and the scalar
    or default vector kernel; other vector tunings are refused."""
    for eq in ("poly2", "product"):
        for dt in ("fp64", "fp32_dev"):
            cfg = _cfg(lbm, shape=(256, 8), dtype=dt, equilibrium=eq)
            ref = lbm.lbm_workspace_bytes(_cfg(lbm, shape=(256, 8), dtype=dt))
            assert lbm.lbm_workspace_bytes(cfg) == ref > 0
            assert lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(64, 4, -1, 1, 0)) > 0
        f32 = _cfg(lbm, shape=(256, 8), dtype="fp32_dev", equilibrium=eq)
        assert lbm.lbm_workspace_bytes(f32, lbm.make_tuning(64, 4, -1, 4, 3)) > 0
        assert lbm.lbm_workspace_bytes(f32, lbm.make_tuning(64, 4, -1, 2, -1)) == 0
        assert lbm.lbm_workspace_bytes(f32, lbm.make_tuning(64, 4, -1, 4, 1)) == 0
        f64 = _cfg(lbm, shape=(256, 8), dtype="fp64", equilibrium=eq)
        assert lbm.lbm_workspace_bytes(f64, lbm.make_tuning(64, 4, -1, 2, 0)) == 0
        # pool slots run the entropic equilibrium only
        assert lbm.lbm_pool_slot_bytes(f64) == 0
        assert b"entropic" in lbm.load_library().lbm_last_error()


def test_d1q3_configs(lbm):
    for dt in ("fp64", "fp32_dev", "fp32_dev_mixed", "fp32_dev_f32"):
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(300,), dtype=dt)) > 0
    for eq in ("entropic", "poly2", "product"):
        assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(512,), dtype="fp32_dev", equilibrium=eq)) > 0
    # vector kernels: 4 floats or 2 doubles per thread when nx tiles evenly
    assert lbm.lbm_workspace_bytes(_cfg(lbm, lattice=3, shape=(256,), dtype="fp32_dev"),
                                   lbm.make_tuning(64, 1, -1, 4, 3)) > 0
    # pool slots run D2Q9 or D3Q27
    assert lbm.lbm_pool_slot_bytes(_cfg(lbm, lattice=3, shape=(64,))) == 0


def test_vn_argument_checks(lbm):
    lib = lbm.load_library()
    E = lbm.LBM_EINVAL
    assert lib.lbm_vn_spectra(27, 0, 0, 256, 1, None, None, None, None, None) == E  # D3Q27 not offered
    assert lib.lbm_vn_spectra(9, 3, 0, 256, 1, None, None, None, None, None) == E
    assert lib.lbm_vn_spectra(9, 0, 2, 256, 1, None, None, None, None, None) == E
    assert lib.lbm_vn_spectra(9, 0, 0, None, 1, None, None, None, None, None) == E
    assert lib.lbm_vn_spectra(9, 0, 0, 256, -1, None, None, None, None, None) == E
    assert lib.lbm_vn_spectra(3, 1, 1, 256, 0, None, None, None, None, None) == lbm.LBM_OK  # nothing to do
    assert lib.lbm_vn_max_radius(9, 0, 0, 256, 4, 0, 256, 256, 256, None) == E  # nk < 1
    assert lib.lbm_vn_max_radius(9, 0, 0, 256, 4, 33, 256, 260, 256, None) == E  # misaligned scratch
    assert lib.lbm_vn_max_radius(9, 0, 0, 256, 4, 33, 256, 256, None, None) == E
    assert lib.lbm_vn_max_radius(9, 0, 0, None, 4, 33, 256, 256, 256, None) == E
    assert lib.lbm_vn_max_radius(1, 0, 0, 256, 4, 33, 256, 256, 256, None) == E


def test_energy_history_null_handle(lbm):
    lib = lbm.load_library()
    assert lib.lbm_energy_history(None, 10, 10, None, 1.0, 256) == lbm.LBM_EINVAL


def test_create_argument_checks_precede_gpu_work(lbm):
    lib = lbm.load_library()
    cfg = _cfg(lbm)
    h = ctypes.c_void_p()
    # NULL workspace / fields / out: rejected on the host
    assert lib.lbm_create(ctypes.byref(cfg), None, 1 << 30, 8, 8, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_create(ctypes.byref(cfg), 256, 1 << 30, None, 8, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_create(ctypes.byref(cfg), 256, 1 << 30, 8, 8, None, None) == lbm.LBM_EINVAL
    # workspace too small or misaligned
    assert lib.lbm_create(ctypes.byref(cfg), 256, 16, 8, 8, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_create(ctypes.byref(cfg), 260, 1 << 30, 8, 8, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert h.value is None
    # NULL handle
    assert lib.lbm_step(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_moments(None, None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_get_populations(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_state_bytes(None) == 0
    assert lib.lbm_save_state(None, 256, 0) == lbm.LBM_EINVAL
    assert lib.lbm_load_state(None, 256, 0, 0) == lbm.LBM_EINVAL
    assert lib.lbm_energy(None, None, 1.0, 256) == lbm.LBM_EINVAL
    assert lib.lbm_destroy(None) == lbm.LBM_OK
    assert b"NULL" in lib.lbm_last_error()


def test_product_package_never_touches_the_oracle():
    pkg = os.path.join(ROOT, "paper_2303_08163_amd")
    for dirpath, _, files in os.walk(pkg):
        for fn in files:
            if fn.endswith((".py", ".hip", ".hpp", ".h", ".cpp")):
                text = open(os.path.join(dirpath, fn)).read()
                assert not re.search(r"^\s*(import|from)\s+oracle\b", text, flags=re.M), fn
                assert "lbm_oracle" not in text and "liblbm_oracle" not in text, fn
    for fn in os.listdir(os.path.join(ROOT, "oracle")):
        if fn.endswith((".py", ".c", ".h")):
            text = open(os.path.join(ROOT, "oracle", fn)).read()
            assert "paper_2303_08163_amd" not in text and "lbm.h" not in text, fn


def test_pool_host_logic(lbm):
    lib = lbm.load_library()
    assert lbm.lbm_pool_table_bytes(0) == 0 and lbm.lbm_pool_table_bytes(65537) == 0
    t16 = lbm.lbm_pool_table_bytes(16)
    assert t16 > 0 and t16 % 256 == 0 and lbm.lbm_pool_table_bytes(32) > t16
    cfg = _cfg(lbm)
    # a slot occupies exactly one domain workspace with the pool's tile
    assert lbm.lbm_pool_slot_bytes(cfg) == lbm.lbm_workspace_bytes(cfg, lbm.make_tuning(64, 4, -1, 1, 0))
    assert lbm.lbm_pool_slot_bytes(_cfg(lbm, tau=0.5)) == 0
    for bad in [dict(tile_x=48, tile_y=4), dict(tile_x=64, tile_y=8), dict(persistent=2), dict(workgroups=-1),
                dict(layout=5), dict(flat=2), dict(flat=-1), dict(row_fit=2), dict(row_fit=-1),
                dict(row_fit=1, flat=1), dict(time_block=3), dict(time_block=-1)]:
        assert lbm.lbm_pool_slot_bytes(cfg, lbm.make_pool_tuning(**bad)) == 0, bad
    # two steps per launch changes the launches only, not a slot's memory
    assert lbm.lbm_pool_slot_bytes(cfg, lbm.make_pool_tuning(time_block=2)) == lbm.lbm_pool_slot_bytes(cfg)
    # the tile-ordered persistent form keeps one 8-byte counter per two-step tile after the
    # buffers of D2Q9 FP64 and FP32-deviation slots (rounded up to 256 bytes): FP64 column
    # tiles of 128 x 64; FP32 in 1024-thread workgroups, whole-row tiles of 16-row sub-tiles
    # (row 300 -> 320 lanes, three sub-tiles) or column tiles of 1024 x 16
    to = lbm.make_pool_tuning(time_block=2, persistent=1)
    for kw, extra in [(dict(shape=(300, 1000)), 256 * 2),  # 3 x 16 tiles: 384 bytes
                      (dict(shape=(300, 1000), dtype="fp32_dev"), 256),  # 21 tiles of 48 rows
                      (dict(shape=(600, 1000), dtype="fp32_dev"), 256 * 2),  # rows of 640 lanes: 63 tiles
                      (dict(shape=(1500, 1000), dtype="fp32_dev"), 256 * 4),  # 2 x 63 column tiles of 1024
                      (dict(), 256),  # 1 x 2 tiles
                      (dict(shape=(300, 1000), dtype="fp32_dev_mixed"), 0),
                      (dict(lattice=27, shape=(16, 16, 16), dtype="fp32_dev"), 0)]:
        c = _cfg(lbm, **kw)
        assert lbm.lbm_pool_slot_bytes(c, to) == lbm.lbm_pool_slot_bytes(c) + extra, kw
    # row fit changes the thread mapping only, not a slot's memory
    assert lbm.lbm_pool_slot_bytes(cfg, lbm.make_pool_tuning(row_fit=1)) == lbm.lbm_pool_slot_bytes(cfg)
    h = ctypes.c_void_p()
    assert lib.lbm_pool_create(4, None, None, 1 << 30, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_pool_create(0, None, 256, 1 << 30, None, ctypes.byref(h)) == lbm.LBM_EINVAL
    assert lib.lbm_pool_create(4, None, 256, 1024, None, ctypes.byref(h)) == lbm.LBM_EINVAL  # arena too small
    assert lib.lbm_pool_create(4, None, 260, 1 << 30, None, ctypes.byref(h)) == lbm.LBM_EINVAL  # misaligned
    assert h.value is None
    slot = ctypes.c_int32()
    n = ctypes.c_int32()
    assert lib.lbm_pool_admit(None, ctypes.byref(cfg), 8, 8, 1, ctypes.byref(slot)) == lbm.LBM_EINVAL
    assert lib.lbm_pool_run(None, 1) == lbm.LBM_EINVAL
    assert lib.lbm_pool_poll(None, None, 0, ctypes.byref(n)) == lbm.LBM_EINVAL
    assert lib.lbm_pool_moments(None, 0, None, None, None) == lbm.LBM_EINVAL
    assert lib.lbm_pool_release(None, 0) == lbm.LBM_EINVAL
    assert lib.lbm_pool_stats_get(None, None) == lbm.LBM_EINVAL
    assert lib.lbm_pool_destroy(None) == lbm.LBM_OK


def test_slab_configs(lbm):
    """z-slabs: two halo planes per population buffer, packed faces of 9 nx ny
    stored values, and the configurations a slab refuses."""
    nx, ny, nz = 70, 5, 4
    for dtype, s in (("fp64", 8), ("fp32_dev", 4)):
        per = lbm.make_config(27, (nx, ny, nz), 0.6, dtype)
        slab = lbm.make_config(27, (nx, ny, nz), 0.6, dtype, z_halo=True)
        plane_bytes = 27 * 80 * ny * s  # rows of 27 runs of pitch 80
        grow = lbm.lbm_workspace_bytes(slab) - lbm.lbm_workspace_bytes(per)
        assert 2 * 2 * plane_bytes <= grow <= 2 * 2 * plane_bytes + 2 * 256
        assert lbm.lbm_halo_bytes(slab) == 9 * nx * ny * s
        assert lbm.lbm_halo_bytes(per) == 0
    assert lbm.lbm_workspace_bytes(lbm.make_config(9, (64, 32), 0.6, "fp64", z_halo=True)) == 0
    assert lbm.lbm_workspace_bytes(lbm.make_config(3, (64,), 0.6, "fp64", z_halo=True)) == 0
    bad = lbm.make_config(27, (8, 8, 8), 0.6, "fp64")
    bad.z_halo = 2
    assert lbm.lbm_workspace_bytes(bad) == 0
    bad = lbm.make_config(27, (8, 8, 8), 0.6, "fp64")
    bad.reserved = 1
    assert lbm.lbm_workspace_bytes(bad) == 0
    slab = lbm.make_config(27, (8, 8, 8), 0.6, "fp64", z_halo=True)
    planes = lbm.make_tuning(layout=lbm.LBM_LAYOUT_PLANES)
    assert lbm.lbm_workspace_bytes(slab, planes) == 0
    assert lbm.lbm_pool_slot_bytes(slab) == 0
    lib = lbm.load_library()
    assert lib.lbm_halo_pack(None, 256, 512) == lbm.LBM_EINVAL
    assert lib.lbm_halo_unpack(None, 256, None) == lbm.LBM_EINVAL
    assert lib.lbm_step_halo(None, 256, 512, 768, 1024) == lbm.LBM_EINVAL


def test_c_abi_demo_compiles_and_links(tmp_path):
    """The plain-C caller (tests/c/abi_demo.c) builds with gcc -std=c99 -Werror
    against include/lbm.h and links against the library (run by a GPU test)."""
    import subprocess
    import __graft_entry__ as entry
    out = str(tmp_path / "abi_demo")
    r = subprocess.run(entry.c_demo_command(out), capture_output=True, text=True)
    assert r.returncode == 0, r.stderr
    assert os.path.exists(out)
