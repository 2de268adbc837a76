"""Dissipation of isothermal pressure waves: the effective viscosity of the
scheme as a function of a uniform convection speed U0 (Sec. "Validation via
dissipation of isothermal pressure waves").

A periodic domain starts from f = f^eq(rho, u) with rho = rho0 + drho sin(2 pi x / nx)
and u = (U0, 0, 0).  In linear acoustics with losses the quadratic energy
E = sum [rho0 |u - U0|^2 / 2 + c_s^2 (rho - rho0)^2 / (2 rho0)] decays as
exp(-((D+1)/D nu + eta/rho) k^2 t) with k = 2 pi / nx; with the LBGK bulk
viscosity eta = (D-1)/D rho nu the bracket is 2 nu for every D, so the
least-squares slope of log E(t) gives nu_eff = -slope / (2 k^2).  Without the
bulk correction nu_eff / nu follows A(U0); with it, it returns close to 1.

Every step and every energy reduction runs in the library's kernels; the
energy history is recorded on the device (lbm_energy_history: the whole run in one call)
and read once, so the host does not synchronise inside the run.  Only the
final log-linear fit runs on the host.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm, workloads

NU_PER_TAU = 1.0 / 3.0  # nu = (tau - 1/2) c_s^2 with c_s^2 = 1/3


def nu_of_tau(tau: float) -> float:
    return (tau - 0.5) * NU_PER_TAU


def wave_fields(nx: int, drho: float, U0: float, rho0: float = 1.0, dim: int = 1, width: int = 1):
    """Initial fields of the wave on a D1Q3 (nx), D2Q9 (width x nx) or D3Q27
    (width x width x nx) grid; the wave runs along x."""
    if dim == 1:
        return workloads.pressure_wave(nx, drho, U0, rho0)
    if dim == 2:
        return workloads.pressure_wave(nx, drho, U0, rho0, ny=width)
    return workloads.pressure_wave(nx, drho, U0, rho0, ny=width, nz=width)


def energy_history(nx: int, drho: float, U0: float, tau: float, steps: int, every: int = 10,
                   dtype: str = "fp64", bulk_correction: bool = False, equilibrium: str = "entropic",
                   dim: int = 1, width: int = 1, rho0: float = 1.0, device="cuda:0"):
    """Run the wave for `steps` steps and return (t, E(t)) sampled every
    `every` steps (t = 0 included), plus the run's final diagnostics."""
    if steps % every:
        raise ValueError("steps must be a multiple of every")
    rho, u = wave_fields(nx, drho, U0, rho0, dim, width)
    U = [U0] + [0.0] * (dim - 1)
    n = steps // every
    with lbm.Domain(rho, u, tau, dtype=dtype, bulk_correction=bulk_correction, rho0=rho0,
                    equilibrium=equilibrium, device=device) as d:
        hist = d.energy_history(steps, every, U, rho0)
        _, _, diag = d.moments(fields=False)  # synchronises; raises on a domain error
        E = hist.cpu().numpy()
    return np.arange(n + 1, dtype=np.int64) * every, E, diag


def decay_rate(t, E, t_min: int) -> float:
    """-slope of the least-squares line through (t, log E) for t >= t_min."""
    t = np.asarray(t, dtype=np.float64)
    E = np.asarray(E, dtype=np.float64)
    sel = t >= t_min
    if sel.sum() < 2 or np.any(E[sel] <= 0):
        raise ValueError("need at least two positive energies in the fit window")
    return -float(np.polyfit(t[sel], np.log(E[sel]), 1)[0])


def effective_viscosity(rate: float, nx: int) -> float:
    k = 2.0 * math.pi / nx
    return rate / (2.0 * k * k)


def sweep(U0s, nx: int = 64, tau: float = 0.65, drho: float = 1e-3, steps: int = 2000, every: int = 10,
          t_min: int = 200, equilibria=("entropic", "product"), corrections=(False, True),
          dtype: str = "fp64", dim: int = 1, width: int = 1):
    """Effective viscosity for every (equilibrium, correction, U0).

    Returns a list of dicts with nu_eff, ratio = nu_eff / nu and
    normalised = nu_eff / nu_eff(U0 = 0) of the same variant (the U0 = 0 run is
    added when absent; it removes the O(k^2) lattice dispersion of the fit)."""
    nu = nu_of_tau(tau)
    grid = sorted(set(float(v) for v in U0s) | {0.0})
    out = []
    for eq in equilibria:
        for corr in corrections:
            rows = []
            for U0 in grid:
                t, E, _ = energy_history(nx, drho, U0, tau, steps, every, dtype, corr, eq, dim, width)
                nu_eff = effective_viscosity(decay_rate(t, E, t_min), nx)
                rows.append(dict(equilibrium=eq, bulk_correction=bool(corr), U0=U0, nu=nu, nu_eff=nu_eff,
                                 ratio=nu_eff / nu))
            base = next(r["nu_eff"] for r in rows if r["U0"] == 0.0)
            for r in rows:
                r["normalised"] = r["nu_eff"] / base
            out.extend(rows)
    return out
