"""Plain FP64 CPU oracle for entropic-equilibrium lattice-BGK (arXiv:2303.08163).

TEST INFRASTRUCTURE ONLY.  The oracle is what the GPU library is checked
against.  Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg
of ``bench.py`` may import it; the product package never does, and the two
share no code.  The arithmetic lives in ``lbm_oracle.c`` (plain C, FP64,
``-O2 -ffp-contract=off``, optional OpenMP over nodes); this module builds it
with gcc and marshals numpy arrays through ctypes.

Field layout everywhere: ``rho`` has the grid's shape (x fastest, i.e. numpy
shape ``(nz, ny, nx)`` in 3-D, ``(ny, nx)`` in 2-D, ``(nx,)`` in 1-D) and ``u``
has shape ``(D, *grid)``.

Parity status: every function here is pinned by tests in
``tests/test_oracle_*.py`` (conservation, entropy minimisation by brute force,
closed forms printed in the paper, low-Mach limits, shear-wave viscosity,
symmetries and embeddings); none is "parity unpinned".  The collision
Jacobian and the von Neumann analysis built on it (``oracle.stability``) are
pinned in ``tests/test_oracle_stability.py`` (finite differences, collision
invariants, the k = 0 spectrum, sound speeds and dissipation at k -> 0, and
the stability limits printed in the paper).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.c")
_LIB_PATH = os.path.join(_HERE, "liblbm_oracle.so")

EQ_KINDS = {"entropic": 0, "poly2": 1, "product": 2}
CORR_MODES = {"off": 0, False: 0, None: 0, "min": 1, True: 1, "product": 2}

_lib = None


def build(verbose: bool = False) -> str:
    """Compile the oracle with gcc (plain FP64, no fast-math, FMA contraction off)."""
    tmp = _LIB_PATH + ".tmp"
    cmd = ["gcc", "-O2", "-ffp-contract=off", "-fno-fast-math", "-fopenmp", "-std=c99",
           "-Wall", "-shared", "-fPIC", _SRC, "-o", tmp, "-lm"]
    if verbose:
        print(" ".join(cmd))
    subprocess.run(cmd, check=True)
    os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH) or os.path.getmtime(_LIB_PATH) < os.path.getmtime(_SRC):
        build()
    lib = ctypes.CDLL(_LIB_PATH)
    dp = ctypes.POINTER(ctypes.c_double)
    ip = ctypes.POINTER(ctypes.c_int)
    lp = ctypes.POINTER(ctypes.c_long)
    lib.oracle_lattice.argtypes = [ctypes.c_int, ip, dp]
    lib.oracle_lattice.restype = ctypes.c_int
    lib.oracle_equilibrium.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_double, dp, dp]
    lib.oracle_equilibrium.restype = ctypes.c_int
    lib.oracle_bulk_A.argtypes = [ctypes.c_int, ctypes.c_double]
    lib.oracle_bulk_A.restype = ctypes.c_double
    lib.oracle_beta.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, dp]
    lib.oracle_beta.restype = ctypes.c_double
    lib.oracle_run.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                               ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp,
                               ctypes.c_long, dp, dp, dp]
    lib.oracle_run.restype = ctypes.c_long
    lib.oracle_run_sample.argtypes = [ctypes.c_int, ctypes.c_long, ctypes.c_long, ctypes.c_long,
                                      ctypes.c_double, ctypes.c_int, ctypes.c_int, dp, dp,
                                      ctypes.c_long, ctypes.c_long, lp, lp, lp, dp, dp]
    lib.oracle_run_sample.restype = ctypes.c_long
    lib.oracle_jacobian.argtypes = [ctypes.c_int, ctypes.c_int, ctypes.c_int, ctypes.c_double, ctypes.c_double,
                                    dp, dp]
    lib.oracle_jacobian.restype = ctypes.c_int
    lib.oracle_set_threads.argtypes = [ctypes.c_int]
    lib.oracle_set_threads.restype = ctypes.c_int
    _lib = lib
    return lib


def _dptr(a: np.ndarray):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _grid3(shape):
    """numpy grid shape (x fastest) -> (D, nx, ny, nz)."""
    D = len(shape)
    if D == 1:
        return 1, shape[0], 1, 1
    if D == 2:
        return 2, shape[1], shape[0], 1
    if D == 3:
        return 3, shape[2], shape[1], shape[0]
    raise ValueError("grid must be 1-, 2- or 3-dimensional")


def set_threads(n: int = 0) -> int:
    """Set the oracle's OpenMP thread count (n <= 0 keeps it); returns the count in effect."""
    return int(_load().oracle_set_threads(int(n)))


def lattice(D: int):
    """Velocities (Q, D) int array and weights (Q,) of the D-dimensional first-neighbour lattice."""
    c = np.zeros((27, 3), dtype=np.intc)
    w = np.zeros(27)
    Q = _load().oracle_lattice(D, c.ctypes.data_as(ctypes.POINTER(ctypes.c_int)), _dptr(w))
    if Q < 0:
        raise ValueError(f"unsupported dimension {D}")
    return c[:Q, :D].copy(), w[:Q].copy()


def equilibrium(rho: float, u, kind: str = "entropic"):
    """Equilibrium populations (Q,) at one node, oracle ordering; also returns the domain flag."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    D = u.shape[0]
    feq = np.zeros(27)
    bad = _load().oracle_equilibrium(D, EQ_KINDS[kind], float(rho), _dptr(u), _dptr(feq))
    if bad < 0:
        raise ValueError("bad arguments")
    return feq[: 3 ** D].copy(), bool(bad)


def bulk_A(u: float, kind: str = "entropic") -> float:
    """Effective-viscosity factor A(u) of a 1-D velocity."""
    return _load().oracle_bulk_A(EQ_KINDS[kind], float(u))


def jacobian(tau: float, u, corr="off", kind: str = "entropic", rho: float = 1.0) -> np.ndarray:
    """Jacobian (Q, Q) of the collision operator at f = f^eq(rho, u), oracle ordering."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    D = u.shape[0]
    J = np.zeros(27 * 27)
    Q = _load().oracle_jacobian(D, EQ_KINDS[kind], CORR_MODES[corr], float(tau), float(rho), _dptr(u), _dptr(J))
    if Q < 0:
        raise ValueError("bad arguments")
    return J[: Q * Q].reshape(Q, Q).copy()


def beta(tau: float, u, corr="off", kind: str = "entropic") -> float:
    """Relaxation frequency beta at a node with velocity u (collision uses 2 beta)."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    return _load().oracle_beta(u.shape[0], EQ_KINDS[kind], CORR_MODES[corr], float(tau), _dptr(u))


def run(rho0, u0, tau: float, steps: int, corr="off", kind: str = "entropic",
        return_f: bool = False, threads: int | None = None):
    """Step the periodic grid `steps` times from f = f^eq(rho0, u0).

    Returns (rho, u, bad) — bad = number of (node, step) pairs out of the
    equilibrium's domain — and f (Q, *grid) when return_f is set.
    """
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    D, nx, ny, nz = _grid3(rho0.shape)
    if u0.shape != (D,) + rho0.shape:
        raise ValueError("u0 must have shape (D, *rho0.shape)")
    rho = np.zeros_like(rho0)
    u = np.zeros_like(u0)
    f = np.zeros((3 ** D,) + rho0.shape) if return_f else None
    if threads is not None:
        set_threads(threads)
    bad = _load().oracle_run(D, nx, ny, nz, float(tau), EQ_KINDS[kind], CORR_MODES[corr],
                             _dptr(rho0), _dptr(u0), int(steps), _dptr(rho), _dptr(u),
                             _dptr(f) if return_f else None)
    if bad < 0:
        raise ValueError("oracle_run: bad arguments or out of memory")
    if return_f:
        return rho, u, int(bad), f
    return rho, u, int(bad)


def run_sample(rho0, u0, tau: float, steps: int, points, corr="off", kind: str = "entropic"):
    """Moments after `steps` steps at sample nodes only.

    points: (S, D) integer array of node coordinates (x, y, z order).
    Returns rho (S,) and u (D, S).
    """
    rho0 = np.ascontiguousarray(rho0, dtype=np.float64)
    u0 = np.ascontiguousarray(u0, dtype=np.float64)
    D, nx, ny, nz = _grid3(rho0.shape)
    pts = np.asarray(points, dtype=np.int64).reshape(-1, D)
    S = pts.shape[0]
    cols = [np.ascontiguousarray(pts[:, a], dtype=np.int64) if a < D else np.zeros(S, np.int64)
            for a in range(3)]
    lp = ctypes.POINTER(ctypes.c_long)
    rho_s = np.zeros(S)
    u_s = np.zeros((D, S))
    rc = _load().oracle_run_sample(D, nx, ny, nz, float(tau), EQ_KINDS[kind], CORR_MODES[corr],
                                   _dptr(rho0), _dptr(u0), int(steps), S,
                                   cols[0].ctypes.data_as(lp), cols[1].ctypes.data_as(lp),
                                   cols[2].ctypes.data_as(lp), _dptr(rho_s), _dptr(u_s))
    if rc < 0:
        raise ValueError("oracle_run_sample: bad arguments or out of memory")
    return rho_s, u_s


def diagnostics(rho, u, rho0: float = 1.0) -> dict:
    """Whole-grid diagnostics of moment fields: mass, momentum, kinetic energy,
    max |u_alpha|, min rho.  Plain numpy sums in FP64."""
    rho = np.asarray(rho, dtype=np.float64)
    u = np.asarray(u, dtype=np.float64)
    D = u.shape[0]
    mom = [float(np.sum(rho * u[a])) for a in range(D)] + [0.0] * (3 - D)
    return {
        "mass": float(np.sum(rho)),
        "momentum": mom,
        "kinetic_energy": float(np.sum(0.5 * rho * np.sum(u * u, axis=0))),
        "max_abs_u": float(np.max(np.abs(u))),
        "min_rho": float(np.min(rho)),
    }
