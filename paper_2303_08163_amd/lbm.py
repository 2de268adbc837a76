"""Python binding of the C ABI in ``include/lbm.h`` (argument marshalling only).

Every function here has the name of the C entry point it wraps and does nothing
but convert arguments, call the native library and turn a negative status into
an exception.  All arithmetic of the method runs in the library's HIP kernels;
there is no Python or CPU fallback: if the built library is missing, loading
fails with an error.

``Domain`` is a convenience owner of one domain's device memory: it allocates
the workspace and the initial fields as torch CUDA tensors (torch is used for
device memory and streams only) and calls the functions above.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm_entropic.so")

# status codes (enum lbm_status)
LBM_OK, LBM_EINVAL, LBM_EDOMAIN, LBM_EDEVICE, LBM_ENOMEM, LBM_EBUSY = 0, -1, -2, -3, -4, -5
LBM_D1Q3, LBM_D2Q9, LBM_D3Q27 = 3, 9, 27
LATTICE_OF_DIM = {1: LBM_D1Q3, 2: LBM_D2Q9, 3: LBM_D3Q27}
LBM_FP64, LBM_FP32_DEV, LBM_FP32_DEV_MIXED, LBM_FP32_DEV_F32 = 0, 1, 2, 3
LBM_EQ_ENTROPIC, LBM_EQ_POLY2, LBM_EQ_PRODUCT = 0, 1, 2
EQUILIBRIA = {"entropic": LBM_EQ_ENTROPIC, "poly2": LBM_EQ_POLY2, "product": LBM_EQ_PRODUCT}

LBM_KERNEL_NODE, LBM_KERNEL_VECTOR, LBM_KERNEL_TWO_STEP, LBM_KERNEL_MULTI_STEP = 1, 2, 3, 4
KERNEL_NAMES = {1: "node", 2: "vector", 3: "two_step", 4: "multi_step"}

DTYPES = {"fp64": LBM_FP64, "fp32_dev": LBM_FP32_DEV, "fp32_dev_mixed": LBM_FP32_DEV_MIXED,
          "fp32_dev_f32": LBM_FP32_DEV_F32}


class lbm_config(ctypes.Structure):
    _fields_ = [("lattice", ctypes.c_int32), ("dtype", ctypes.c_int32),
                ("nx", ctypes.c_int64), ("ny", ctypes.c_int64), ("nz", ctypes.c_int64),
                ("tau", ctypes.c_double), ("bulk_correction", ctypes.c_int32),
                ("equilibrium", ctypes.c_int32), ("rho0", ctypes.c_double),
                ("z_halo", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lbm_tuning(ctypes.Structure):
    _fields_ = [("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("plane_pad", ctypes.c_int32), ("nodes_per_thread", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("layout", ctypes.c_int32), ("time_block", ctypes.c_int32),
                ("time_rows", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class lbm_diag(ctypes.Structure):
    _fields_ = [("mass", ctypes.c_double), ("momentum", ctypes.c_double * 3),
                ("kinetic_energy", ctypes.c_double), ("max_abs_u", ctypes.c_double),
                ("min_rho", ctypes.c_double), ("steps", ctypes.c_int64),
                ("domain_error", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {"mass": self.mass, "momentum": list(self.momentum),
                "kinetic_energy": self.kinetic_energy, "max_abs_u": self.max_abs_u,
                "min_rho": self.min_rho, "steps": int(self.steps),
                "domain_error": bool(self.domain_error)}


class lbm_launch_info(ctypes.Structure):
    _fields_ = [("kernel", ctypes.c_int32), ("nodes_per_thread", ctypes.c_int32), ("row_wave", ctypes.c_int32),
                ("flags", ctypes.c_int32), ("block_x", ctypes.c_int32), ("block_y", ctypes.c_int32),
                ("layout", ctypes.c_int32), ("time_block", ctypes.c_int32), ("time_cols", ctypes.c_int32),
                ("time_rows", ctypes.c_int32), ("graph_steps", ctypes.c_int32), ("reserved", ctypes.c_int32)]

    def as_dict(self) -> dict:
        d = {k: getattr(self, k) for k, _ in self._fields_ if k != "reserved"}
        d["kernel"] = KERNEL_NAMES.get(d["kernel"], d["kernel"])
        return d


class lbm_pool_tuning(ctypes.Structure):
    _fields_ = [("tile_x", ctypes.c_int32), ("tile_y", ctypes.c_int32), ("persistent", ctypes.c_int32),
                ("workgroups", ctypes.c_int32), ("layout", ctypes.c_int32), ("flat", ctypes.c_int32),
                ("row_fit", ctypes.c_int32), ("time_block", ctypes.c_int32), ("time_rows", ctypes.c_int32),
                ("spin_log2", ctypes.c_int32)]


class lbm_pool_stats(ctypes.Structure):
    _fields_ = [("max_slots", ctypes.c_int32), ("used_slots", ctypes.c_int32),
                ("arena_bytes", ctypes.c_int64), ("free_bytes", ctypes.c_int64),
                ("largest_free_block", ctypes.c_int64), ("runs", ctypes.c_int64), ("launches", ctypes.c_int64)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class lbm_slot_info(ctypes.Structure):
    _fields_ = [("used", ctypes.c_int32), ("finished", ctypes.c_int32), ("steps_done", ctypes.c_int64),
                ("steps_remaining", ctypes.c_int64), ("bytes", ctypes.c_int64), ("domain_error", ctypes.c_int32),
                ("device_error", ctypes.c_int32)]

    def as_dict(self) -> dict:
        return {k: getattr(self, k) for k, _ in self._fields_}


class LBMError(RuntimeError):
    def __init__(self, status: int, where: str, message: str = ""):
        self.status = status
        super().__init__(f"{where}: {lbm_status_string(status)}" + (f" ({message})" if message else ""))


class LBMDomainError(LBMError):
    """A node left rho > 0, |u_alpha| < 1 (outputs were still written)."""


_lib = None

# Exported symbols the header declares (checked by the CPU test suite).
EXPORTS = ("lbm_workspace_bytes", "lbm_workspace_bytes_tuned", "lbm_create", "lbm_create_tuned",
           "lbm_step", "lbm_moments", "lbm_get_populations", "lbm_energy", "lbm_energy_history", "lbm_destroy", "lbm_status_string",
           "lbm_last_error", "lbm_version", "lbm_pool_table_bytes", "lbm_pool_slot_bytes", "lbm_pool_create",
           "lbm_pool_admit", "lbm_pool_run", "lbm_pool_poll", "lbm_pool_moments", "lbm_pool_get_populations",
           "lbm_pool_release", "lbm_pool_stats_get", "lbm_pool_slot_info", "lbm_pool_destroy",
           "lbm_vn_spectra", "lbm_vn_max_radius", "lbm_halo_bytes", "lbm_halo_pack", "lbm_halo_unpack",
           "lbm_step_halo", "lbm_state_bytes", "lbm_save_state", "lbm_load_state", "lbm_get_launch_info",
           "lbm_pool_admit_async", "lbm_pool_collect", "lbm_ceiling_stream", "lbm_ceiling_copy",
           "lbm_vn_max_radius_noalloc")


def load_library(path: str = LIB_PATH):
    """Load the native library (raises OSError/ImportError when it is not built).

    torch is imported first so that the library binds to the HIP runtime torch
    already loaded (same soname): one runtime per process, so torch's device
    pointers and streams are valid handles for the library."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(path):
        raise ImportError(f"native library {path} is not built; run __graft_entry__.build()")
    try:
        import torch  # noqa: F401
    except ImportError:
        pass
    lib = ctypes.CDLL(path)
    vp, sz, i64 = ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int64
    cfgp, tunp = ctypes.POINTER(lbm_config), ctypes.POINTER(lbm_tuning)
    sig = {
        "lbm_workspace_bytes": (sz, [cfgp]),
        "lbm_workspace_bytes_tuned": (sz, [cfgp, tunp]),
        "lbm_create": (ctypes.c_int, [cfgp, vp, sz, vp, vp, vp, ctypes.POINTER(vp)]),
        "lbm_create_tuned": (ctypes.c_int, [cfgp, tunp, vp, sz, vp, vp, vp, ctypes.POINTER(vp)]),
        "lbm_step": (ctypes.c_int, [vp, i64]),
        "lbm_moments": (ctypes.c_int, [vp, vp, vp, ctypes.POINTER(lbm_diag)]),
        "lbm_get_populations": (ctypes.c_int, [vp, vp]),
        "lbm_get_launch_info": (ctypes.c_int, [vp, ctypes.POINTER(lbm_launch_info)]),
        "lbm_ceiling_stream": (ctypes.c_int, [vp, i64]),
        "lbm_ceiling_copy": (ctypes.c_int, [vp, vp, sz, vp]),
        "lbm_energy": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp]),
        "lbm_energy_history": (ctypes.c_int, [vp, i64, i64, ctypes.POINTER(ctypes.c_double), ctypes.c_double, vp]),
        "lbm_halo_bytes": (sz, [cfgp]),
        "lbm_halo_pack": (ctypes.c_int, [vp, vp, vp]),
        "lbm_halo_unpack": (ctypes.c_int, [vp, vp, vp]),
        "lbm_step_halo": (ctypes.c_int, [vp, vp, vp, vp, vp]),
        "lbm_state_bytes": (sz, [vp]),
        "lbm_save_state": (ctypes.c_int, [vp, vp, sz]),
        "lbm_load_state": (ctypes.c_int, [vp, vp, sz, i64]),
        "lbm_vn_spectra": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, i64, vp, vp, vp, vp,
                                          vp]),
        "lbm_vn_max_radius": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, i64,
                                             ctypes.c_int32, vp, vp, vp, vp]),
        "lbm_vn_max_radius_noalloc": (ctypes.c_int, [ctypes.c_int32, ctypes.c_int32, ctypes.c_int32, vp, i64,
                                                     ctypes.c_int32, vp, vp, vp]),
        "lbm_destroy": (ctypes.c_int, [vp]),
        "lbm_status_string": (ctypes.c_char_p, [ctypes.c_int]),
        "lbm_last_error": (ctypes.c_char_p, []),
        "lbm_version": (ctypes.c_char_p, []),
        "lbm_pool_table_bytes": (sz, [ctypes.c_int32]),
        "lbm_pool_slot_bytes": (sz, [cfgp, ctypes.POINTER(lbm_pool_tuning)]),
        "lbm_pool_create": (ctypes.c_int, [ctypes.c_int32, ctypes.POINTER(lbm_pool_tuning), vp, sz, vp,
                                           ctypes.POINTER(vp)]),
        "lbm_pool_admit": (ctypes.c_int, [vp, cfgp, vp, vp, i64, ctypes.POINTER(ctypes.c_int32)]),
        "lbm_pool_admit_async": (ctypes.c_int, [vp, cfgp, vp, vp, i64, ctypes.POINTER(ctypes.c_int32)]),
        "lbm_pool_run": (ctypes.c_int, [vp, i64]),
        "lbm_pool_collect": (ctypes.c_int, [vp, i64, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                            ctypes.POINTER(ctypes.c_int32)]),
        "lbm_pool_poll": (ctypes.c_int, [vp, ctypes.POINTER(ctypes.c_int32), ctypes.c_int32,
                                         ctypes.POINTER(ctypes.c_int32)]),
        "lbm_pool_moments": (ctypes.c_int, [vp, ctypes.c_int32, vp, vp, ctypes.POINTER(lbm_diag)]),
        "lbm_pool_get_populations": (ctypes.c_int, [vp, ctypes.c_int32, vp]),
        "lbm_pool_release": (ctypes.c_int, [vp, ctypes.c_int32]),
        "lbm_pool_stats_get": (ctypes.c_int, [vp, ctypes.POINTER(lbm_pool_stats)]),
        "lbm_pool_slot_info": (ctypes.c_int, [vp, ctypes.c_int32, ctypes.POINTER(lbm_slot_info)]),
        "lbm_pool_destroy": (ctypes.c_int, [vp]),
    }
    for name, (res, args) in sig.items():
        fn = getattr(lib, name)
        fn.restype = res
        fn.argtypes = args
    _lib = lib
    return lib


def _check(status: int, where: str) -> int:
    if status == LBM_OK:
        return status
    msg = load_library().lbm_last_error().decode()
    if status == LBM_EDOMAIN:
        raise LBMDomainError(status, where, msg)
    raise LBMError(status, where, msg)


def make_config(lattice: int, shape, tau: float, dtype="fp32_dev", bulk_correction=False,
                rho0: float = 1.0, equilibrium="entropic", z_halo=False) -> lbm_config:
    """shape = (nx,) for D1Q3, (nx, ny) for D2Q9 or (nx, ny, nz) for D3Q27 (x first);
    equilibrium: "entropic", "poly2", "product" or an LBM_EQ_* value; z_halo: a
    z-slab of a domain split along z (halo planes instead of the wrap in z)."""
    nx = int(shape[0])
    ny = int(shape[1]) if len(shape) > 1 else 1
    nz = int(shape[2]) if len(shape) > 2 else 1
    return lbm_config(int(lattice), DTYPES.get(dtype, dtype), nx, ny, nz, float(tau),
                      int(bool(bulk_correction)), EQUILIBRIA.get(equilibrium, equilibrium), float(rho0),
                      int(z_halo), 0)


LBM_TUNE_NT_STORE, LBM_TUNE_NT_LOAD = 1, 2
LBM_LAYOUT_DEFAULT, LBM_LAYOUT_ROWS, LBM_LAYOUT_PLANES = 0, 1, 2


def make_tuning(block_x=0, block_y=0, plane_pad=-1, nodes_per_thread=0, flags=-1, layout=0, time_block=0,
                time_rows=0) -> lbm_tuning:
    return lbm_tuning(int(block_x), int(block_y), int(plane_pad), int(nodes_per_thread), int(flags),
                      int(layout), int(time_block), int(time_rows), 0)


def lbm_workspace_bytes(cfg: lbm_config, tuning: lbm_tuning | None = None) -> int:
    lib = load_library()
    if tuning is None:
        return int(lib.lbm_workspace_bytes(ctypes.byref(cfg)))
    return int(lib.lbm_workspace_bytes_tuned(ctypes.byref(cfg), ctypes.byref(tuning)))


def lbm_create(cfg: lbm_config, workspace: int, ws_bytes: int, rho: int, u: int, stream: int = 0,
               tuning: lbm_tuning | None = None) -> ctypes.c_void_p:
    """Pointers are integers (device addresses / hipStream_t); returns the handle."""
    lib = load_library()
    h = ctypes.c_void_p()
    if tuning is None:
        st = lib.lbm_create(ctypes.byref(cfg), workspace, ws_bytes, rho, u, stream, ctypes.byref(h))
    else:
        st = lib.lbm_create_tuned(ctypes.byref(cfg), ctypes.byref(tuning), workspace, ws_bytes, rho, u,
                                  stream, ctypes.byref(h))
    _check(st, "lbm_create")
    return h


def lbm_step(h, nsteps: int) -> None:
    _check(load_library().lbm_step(h, int(nsteps)), "lbm_step")


def lbm_moments(h, rho: int | None, u: int | None, raise_on_domain: bool = True) -> lbm_diag:
    d = lbm_diag()
    st = load_library().lbm_moments(h, rho, u, ctypes.byref(d))
    if st == LBM_EDOMAIN and not raise_on_domain:
        return d
    _check(st, "lbm_moments")
    return d


def lbm_get_populations(h, out: int) -> None:
    _check(load_library().lbm_get_populations(h, out), "lbm_get_populations")


def lbm_get_launch_info(h) -> dict:
    info = lbm_launch_info()
    _check(load_library().lbm_get_launch_info(h, ctypes.byref(info)), "lbm_get_launch_info")
    return info.as_dict()


def lbm_ceiling_stream(h, nsteps: int) -> None:
    _check(load_library().lbm_ceiling_stream(h, int(nsteps)), "lbm_ceiling_stream")


def lbm_ceiling_copy(src: int, dst: int, nbytes: int, stream=None) -> None:
    _check(load_library().lbm_ceiling_copy(src, dst, int(nbytes), stream), "lbm_ceiling_copy")


def lbm_state_bytes(h) -> int:
    return int(load_library().lbm_state_bytes(h))


def lbm_save_state(h, dst: int, nbytes: int) -> None:
    _check(load_library().lbm_save_state(h, dst, nbytes), "lbm_save_state")


def lbm_load_state(h, src: int, nbytes: int, steps: int) -> None:
    _check(load_library().lbm_load_state(h, src, nbytes, steps), "lbm_load_state")


def lbm_halo_bytes(cfg: lbm_config) -> int:
    return int(load_library().lbm_halo_bytes(ctypes.byref(cfg)))


def lbm_halo_pack(h, lower: int | None, upper: int | None) -> None:
    _check(load_library().lbm_halo_pack(h, lower, upper), "lbm_halo_pack")


def lbm_halo_unpack(h, lower: int | None, upper: int | None) -> None:
    _check(load_library().lbm_halo_unpack(h, lower, upper), "lbm_halo_unpack")


def lbm_step_halo(h, recv_lower: int, recv_upper: int, send_lower: int, send_upper: int) -> None:
    _check(load_library().lbm_step_halo(h, recv_lower, recv_upper, send_lower, send_upper), "lbm_step_halo")


def lbm_energy(h, U, rho_ref: float, out: int) -> None:
    """Enqueue E about (rho_ref, U) into the device double at address out."""
    arr = None if U is None else (ctypes.c_double * 3)(*[float(v) for v in U] + [0.0] * (3 - len(U)))
    _check(load_library().lbm_energy(h, arr, float(rho_ref), out), "lbm_energy")


def lbm_energy_history(h, steps: int, every: int, U, rho_ref: float, out: int) -> None:
    """Enqueue steps // every + 1 energies, every `every` steps of a run, into
    the device doubles at address out."""
    arr = None if U is None else (ctypes.c_double * 3)(*[float(v) for v in U] + [0.0] * (3 - len(U)))
    _check(load_library().lbm_energy_history(h, int(steps), int(every), arr, float(rho_ref), out),
           "lbm_energy_history")


def lbm_vn_spectra(lattice: int, equilibrium, bulk_correction, cases: int, count: int, radius, eig, info,
                   flops=None, stream=None) -> None:
    _check(load_library().lbm_vn_spectra(int(lattice), EQUILIBRIA.get(equilibrium, equilibrium),
                                          int(bool(bulk_correction)), cases, int(count), radius, eig, info, flops,
                                          stream), "lbm_vn_spectra")


def lbm_vn_max_radius(lattice: int, equilibrium, bulk_correction, states: int, n_states: int, nk: int,
                      max_radius: int, scratch: int, unconverged: int, stream=None) -> None:
    _check(load_library().lbm_vn_max_radius(int(lattice), EQUILIBRIA.get(equilibrium, equilibrium),
                                             int(bool(bulk_correction)), states, int(n_states), int(nk),
                                             max_radius, scratch, unconverged, stream), "lbm_vn_max_radius")


def lbm_vn_max_radius_noalloc(lattice: int, equilibrium, bulk_correction, states: int, n_states: int, nk: int,
                              max_radius: int, unconverged: int, stream=None) -> None:
    _check(load_library().lbm_vn_max_radius_noalloc(int(lattice), EQUILIBRIA.get(equilibrium, equilibrium),
                                                    int(bool(bulk_correction)), states, int(n_states), int(nk),
                                                    max_radius, unconverged, stream), "lbm_vn_max_radius_noalloc")


def lbm_destroy(h) -> None:
    _check(load_library().lbm_destroy(h), "lbm_destroy")


def make_pool_tuning(tile_x=0, tile_y=0, persistent=0, workgroups=0, layout=0, flat=0,
                     row_fit=0, time_block=0, spin_log2=0, time_rows=0) -> lbm_pool_tuning:
    t = lbm_pool_tuning()
    t.tile_x, t.tile_y, t.persistent, t.workgroups, t.layout, t.flat, t.row_fit, t.time_block = (
        int(tile_x), int(tile_y), int(persistent), int(workgroups), int(layout), int(flat), int(row_fit),
        int(time_block))
    t.spin_log2 = int(spin_log2)
    t.time_rows = int(time_rows)
    return t


def lbm_pool_table_bytes(max_slots: int) -> int:
    return int(load_library().lbm_pool_table_bytes(int(max_slots)))


def lbm_pool_slot_bytes(cfg: lbm_config, tuning: lbm_pool_tuning | None = None) -> int:
    return int(load_library().lbm_pool_slot_bytes(ctypes.byref(cfg), ctypes.byref(tuning) if tuning else None))


def lbm_pool_create(max_slots: int, arena: int, arena_bytes: int, stream: int = 0,
                    tuning: lbm_pool_tuning | None = None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    st = load_library().lbm_pool_create(int(max_slots), ctypes.byref(tuning) if tuning else None, arena,
                                        arena_bytes, stream, ctypes.byref(h))
    _check(st, "lbm_pool_create")
    return h


def lbm_pool_admit(pool, cfg: lbm_config, rho: int, u: int, nsteps: int) -> int:
    """Returns the slot index; raises LBMError (status LBM_EBUSY / LBM_ENOMEM when not admissible)."""
    slot = ctypes.c_int32(-1)
    _check(load_library().lbm_pool_admit(pool, ctypes.byref(cfg), rho, u, int(nsteps), ctypes.byref(slot)),
           "lbm_pool_admit")
    return int(slot.value)


def lbm_pool_admit_async(pool, cfg: lbm_config, rho: int, u: int, nsteps: int) -> int:
    """lbm_pool_admit without the synchronisation; the initial state is checked
    by a later poll or collect."""
    slot = ctypes.c_int32(-1)
    _check(load_library().lbm_pool_admit_async(pool, ctypes.byref(cfg), rho, u, int(nsteps), ctypes.byref(slot)),
           "lbm_pool_admit_async")
    return int(slot.value)


def lbm_pool_run(pool, k: int) -> None:
    _check(load_library().lbm_pool_run(pool, int(k)), "lbm_pool_run")


def lbm_pool_poll(pool, capacity: int = 65536) -> list:
    buf = (ctypes.c_int32 * max(1, capacity))()
    n = ctypes.c_int32(0)
    _check(load_library().lbm_pool_poll(pool, buf, int(capacity), ctypes.byref(n)), "lbm_pool_poll")
    return [int(buf[i]) for i in range(n.value)]


def lbm_pool_collect(pool, after_run: int = 0, capacity: int = 65536) -> list:
    buf = (ctypes.c_int32 * max(1, capacity))()
    n = ctypes.c_int32(0)
    _check(load_library().lbm_pool_collect(pool, int(after_run), buf, int(capacity), ctypes.byref(n)),
           "lbm_pool_collect")
    return [int(buf[i]) for i in range(n.value)]


def lbm_pool_moments(pool, slot: int, rho: int | None, u: int | None, raise_on_domain: bool = True) -> lbm_diag:
    d = lbm_diag()
    st = load_library().lbm_pool_moments(pool, int(slot), rho, u, ctypes.byref(d))
    if st == LBM_EDOMAIN and not raise_on_domain:
        return d
    _check(st, "lbm_pool_moments")
    return d


def lbm_pool_get_populations(pool, slot: int, out: int) -> None:
    _check(load_library().lbm_pool_get_populations(pool, int(slot), out), "lbm_pool_get_populations")


def lbm_pool_release(pool, slot: int) -> None:
    _check(load_library().lbm_pool_release(pool, int(slot)), "lbm_pool_release")


def lbm_pool_stats_get(pool) -> dict:
    st = lbm_pool_stats()
    _check(load_library().lbm_pool_stats_get(pool, ctypes.byref(st)), "lbm_pool_stats_get")
    return st.as_dict()


def lbm_pool_slot_info(pool, slot: int) -> dict:
    info = lbm_slot_info()
    _check(load_library().lbm_pool_slot_info(pool, int(slot), ctypes.byref(info)), "lbm_pool_slot_info")
    return info.as_dict()


def lbm_pool_destroy(pool) -> None:
    _check(load_library().lbm_pool_destroy(pool), "lbm_pool_destroy")


def lbm_status_string(status: int) -> str:
    return load_library().lbm_status_string(int(status)).decode()


def lbm_version() -> str:
    return load_library().lbm_version().decode()


class Domain:
    """One periodic domain on the GPU.

    rho: numpy array of the grid's shape ((nx,), (ny, nx) or (nz, ny, nx), x fastest);
    u: (D, *rho.shape).  The fields are copied to the device as float64.
    stream: a torch.cuda.Stream (default: torch's current stream).
    equilibrium: "entropic" (default), "poly2" or "product" (LBM_EQ_*).
    """

    def __init__(self, rho, u, tau: float, dtype="fp32_dev", bulk_correction=False, rho0: float = 1.0,
                 stream=None, tuning: lbm_tuning | None = None, device="cuda:0", equilibrium="entropic",
                 z_halo: bool = False):
        import torch
        load_library()
        on_device = isinstance(rho, torch.Tensor) and rho.is_cuda
        if not on_device:
            rho = np.asarray(rho, dtype=np.float64)
            u = np.asarray(u, dtype=np.float64)
        D = rho.ndim
        if D not in (1, 2, 3) or tuple(u.shape) != (D,) + tuple(rho.shape):
            raise ValueError("rho must be 1-D, 2-D or 3-D and u of shape (D, *rho.shape)")
        self.shape = tuple(rho.shape)
        self.D = D
        self.lattice = LATTICE_OF_DIM[D]
        self.Q = 3 ** D
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.cfg = make_config(self.lattice, rho.shape[::-1], tau, dtype, bulk_correction, rho0, equilibrium,
                               z_halo)
        self.z_halo = bool(z_halo)
        self.tuning = tuning
        nbytes = lbm_workspace_bytes(self.cfg, tuning)
        if nbytes == 0:
            raise LBMError(LBM_EINVAL, "lbm_workspace_bytes", load_library().lbm_last_error().decode())
        self.ws_bytes = nbytes
        self._ws = torch.empty(nbytes + 256, dtype=torch.uint8, device=self.device)
        base = self._ws.data_ptr()
        self._ws_ptr = (base + 255) // 256 * 256
        if on_device:
            rho_d = rho.to(self.device, torch.float64).contiguous()
            u_d = u.to(self.device, torch.float64).contiguous()
            torch.cuda.current_stream(self.device).synchronize()
        else:
            with torch.cuda.stream(self.stream):
                rho_d = torch.from_numpy(np.ascontiguousarray(rho)).to(self.device)
                u_d = torch.from_numpy(np.ascontiguousarray(u)).to(self.device)
        self.stream.synchronize()
        self.handle = lbm_create(self.cfg, self._ws_ptr, nbytes, rho_d.data_ptr(), u_d.data_ptr(),
                                 self.stream.cuda_stream, tuning)
        del rho_d, u_d

    @classmethod
    def from_device(cls, rho, u, tau: float, **kw):
        """Domain from float64 CUDA tensors already on the device."""
        return cls(rho, u, tau, **kw)

    @property
    def n(self) -> int:
        return int(np.prod(self.shape))

    def step(self, nsteps: int) -> None:
        lbm_step(self.handle, nsteps)

    def step_halo(self, recv_lower, recv_upper, send_lower, send_upper) -> None:
        """One z-slab step with the halo exchange fused into the kernel: reads
        the entering populations from recv_lower / recv_upper (the neighbours'
        outgoing faces) and writes the leaving ones to send_lower /
        send_upper (CUDA tensors of halo_bytes() bytes each)."""
        lbm_step_halo(self.handle, recv_lower.data_ptr(), recv_upper.data_ptr(), send_lower.data_ptr(),
                      send_upper.data_ptr())

    def launch_info(self) -> dict:
        """The launch the library chose for this domain (kernel kind, nodes per
        thread, row-wave form, cache hints, workgroup shape, steps per launch)."""
        return lbm_get_launch_info(self.handle)

    def save_state(self):
        """Checkpoint: a CUDA uint8 tensor holding the stored state (bit-exact),
        and the step count.  Raises LBMDomainError if the domain flag is set."""
        import torch
        n = lbm_state_bytes(self.handle)
        buf = torch.empty(n, dtype=torch.uint8, device=self.device)
        torch.cuda.current_stream(self.device).synchronize()  # buf comes from torch's current stream
        lbm_save_state(self.handle, buf.data_ptr(), n)
        steps = self.moments(fields=False)[2]["steps"]  # synchronises
        return buf, steps

    def load_state(self, buf, steps: int) -> None:
        """Restart from a save_state() checkpoint of a domain with the same
        configuration and tuning."""
        lbm_load_state(self.handle, buf.data_ptr(), buf.numel() * buf.element_size(), int(steps))

    def halo_bytes(self) -> int:
        """Bytes of one packed face of a z-slab (0 for a periodic domain)."""
        return lbm_halo_bytes(self.cfg)

    def halo_pack(self, lower, upper) -> None:
        """Enqueue the outgoing populations of both faces (CUDA tensors of at
        least halo_bytes() bytes, or None to skip a face): plane 0's c_z = -1
        populations into lower, plane nz - 1's c_z = +1 into upper."""
        lbm_halo_pack(self.handle, None if lower is None else lower.data_ptr(),
                      None if upper is None else upper.data_ptr())

    def halo_unpack(self, lower, upper) -> None:
        """Enqueue lower (the slab below's upper pack) into the halo plane
        below plane 0 and upper (the slab above's lower pack) into the halo
        plane above plane nz - 1; None skips a face."""
        lbm_halo_unpack(self.handle, None if lower is None else lower.data_ptr(),
                        None if upper is None else upper.data_ptr())

    def moments(self, fields: bool = True, raise_on_domain: bool = True):
        """(rho, u, diag) with rho, u as numpy float64 arrays (None if fields=False)."""
        import torch
        if not fields:
            return None, None, lbm_moments(self.handle, None, None, raise_on_domain).as_dict()
        rho_d = torch.empty(self.shape, dtype=torch.float64, device=self.device)
        u_d = torch.empty((self.D,) + self.shape, dtype=torch.float64, device=self.device)
        d = lbm_moments(self.handle, rho_d.data_ptr(), u_d.data_ptr(), raise_on_domain)
        return rho_d.cpu().numpy(), u_d.cpu().numpy(), d.as_dict()

    def moments_device(self, rho_d, u_d, raise_on_domain: bool = True) -> dict:
        return lbm_moments(self.handle, rho_d.data_ptr(), u_d.data_ptr(), raise_on_domain).as_dict()

    def populations(self):
        import torch
        out = torch.empty((self.Q,) + self.shape, dtype=torch.float64, device=self.device)
        lbm_get_populations(self.handle, out.data_ptr())
        return out.cpu().numpy()

    def energy(self, U=None, rho_ref: float = 1.0, out=None):
        """Enqueue the acoustic energy about (rho_ref, U) (no synchronisation).

        out: a float64 CUDA tensor element to write (e.g. history[t]); a new
        one-element tensor when None.  Returns the tensor written."""
        import torch
        if out is None:
            out = torch.empty(1, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda:
            raise ValueError("out must be a float64 CUDA tensor")
        lbm_energy(self.handle, U, rho_ref, out.data_ptr())
        return out

    def energy_history(self, steps: int, every: int, U=None, rho_ref: float = 1.0, out=None):
        """Enqueue `steps` steps with the energy recorded before the first and
        after every `every` (no synchronisation).  out: a float64 CUDA tensor
        of steps // every + 1 elements (a new one when None).  Returns it."""
        import torch
        n = steps // every + 1 if every > 0 else 0
        if out is None:
            out = torch.empty(n, dtype=torch.float64, device=self.device)
        if out.dtype != torch.float64 or not out.is_cuda or not out.is_contiguous() or out.numel() < n:
            raise ValueError("out must be a contiguous float64 CUDA tensor of steps // every + 1 elements")
        lbm_energy_history(self.handle, steps, every, U, rho_ref, out.data_ptr())
        return out

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            lbm_destroy(self.handle)
            self.handle = None
            self._ws = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class Pool:
    """A pool of slots on one device arena (a torch uint8 tensor of arena_bytes).

    admit() copies the initial fields (numpy, shapes as for Domain) to the
    device and starts a slot with a step budget; run(k) advances every active
    slot by up to k steps; poll() lists finished slots.
    """

    def __init__(self, arena_bytes: int, max_slots: int = 1024, tuning: lbm_pool_tuning | None = None,
                 stream=None, device="cuda:0"):
        import torch
        load_library()
        self.device = torch.device(device)
        self.stream = stream if stream is not None else torch.cuda.current_stream(self.device)
        self.max_slots = int(max_slots)
        self.tuning = tuning
        self.arena_bytes = int(arena_bytes)
        self._arena = torch.empty(self.arena_bytes + 256, dtype=torch.uint8, device=self.device)
        base = (self._arena.data_ptr() + 255) // 256 * 256
        self.handle = lbm_pool_create(self.max_slots, base, self.arena_bytes, self.stream.cuda_stream, tuning)
        self.shapes = {}
        # Outputs of reads come from torch's allocator on a stream of their own: a
        # read of a finished slot runs on the pool's second stream while later work
        # is still queued on the pool's stream, so its output memory must not be a
        # block that queued work there may still use (torch reuses a block freed on
        # a stream for that stream's next allocation at once).
        self._read_stream = torch.cuda.Stream(self.device)

    def slot_bytes(self, shape, tau=0.6, dtype="fp32_dev", bulk_correction=False, rho0=1.0) -> int:
        lattice = LBM_D2Q9 if len(shape) == 2 else LBM_D3Q27
        return lbm_pool_slot_bytes(make_config(lattice, shape[::-1], tau, dtype, bulk_correction, rho0), self.tuning)

    def admit(self, rho, u, tau: float, nsteps: int, dtype="fp32_dev", bulk_correction=False,
              rho0: float = 1.0) -> int:
        import torch
        rho = np.ascontiguousarray(rho, dtype=np.float64)
        u = np.ascontiguousarray(u, dtype=np.float64)
        D = rho.ndim
        if D not in (2, 3) or u.shape != (D,) + rho.shape:
            raise ValueError("rho must be 2-D or 3-D and u of shape (D, *rho.shape)")
        cfg = make_config(LBM_D2Q9 if D == 2 else LBM_D3Q27, rho.shape[::-1], tau, dtype, bulk_correction, rho0)
        with torch.cuda.stream(self.stream):
            rho_d = torch.from_numpy(rho).to(self.device, non_blocking=False)
            u_d = torch.from_numpy(u).to(self.device, non_blocking=False)
        slot = lbm_pool_admit(self.handle, cfg, rho_d.data_ptr(), u_d.data_ptr(), nsteps)
        self.shapes[slot] = rho.shape
        return slot

    def try_admit(self, *args, **kw):
        """admit(), but None instead of an error when no slot or memory is free."""
        try:
            return self.admit(*args, **kw)
        except LBMError as e:
            if e.status in (LBM_EBUSY, LBM_ENOMEM):
                return None
            raise

    def run(self, k: int) -> None:
        lbm_pool_run(self.handle, k)

    def poll(self) -> list:
        return lbm_pool_poll(self.handle, self.max_slots)

    def moments(self, slot: int, fields: bool = True, raise_on_domain: bool = True):
        import torch
        if not fields:
            return None, None, lbm_pool_moments(self.handle, slot, None, None, raise_on_domain).as_dict()
        shape = self.shapes[slot]
        with torch.cuda.stream(self._read_stream):
            rho_d = torch.empty(shape, dtype=torch.float64, device=self.device)
            u_d = torch.empty((len(shape),) + shape, dtype=torch.float64, device=self.device)
            d = lbm_pool_moments(self.handle, slot, rho_d.data_ptr(), u_d.data_ptr(), raise_on_domain)
            return rho_d.cpu().numpy(), u_d.cpu().numpy(), d.as_dict()

    def populations(self, slot: int):
        import torch
        shape = self.shapes[slot]
        Q = 9 if len(shape) == 2 else 27
        with torch.cuda.stream(self._read_stream):
            out = torch.empty((Q,) + shape, dtype=torch.float64, device=self.device)
            lbm_pool_get_populations(self.handle, slot, out.data_ptr())
            return out.cpu().numpy()

    def release(self, slot: int) -> None:
        lbm_pool_release(self.handle, slot)
        self.shapes.pop(slot, None)

    def stats(self) -> dict:
        return lbm_pool_stats_get(self.handle)

    def slot_info(self, slot: int) -> dict:
        return lbm_pool_slot_info(self.handle, slot)

    def close(self) -> None:
        if getattr(self, "handle", None) is not None:
            lbm_pool_destroy(self.handle)
            self.handle = None
            self._arena = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
