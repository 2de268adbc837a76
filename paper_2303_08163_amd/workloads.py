"""Seeded synthetic inputs: initial density and velocity fields, batch and
request mixes.

This module holds no part of the method's arithmetic (no equilibrium, no
collision, no streaming): it only writes the initial macroscopic fields
(rho, u) that both the GPU library and the CPU oracle start from, plus the
seeded parameter draws of the batched and serving workloads.  It imports
nothing from the rest of the package.

The paper runs no public dataset; its numerical experiments are analytic
periodic flows (Sec. "Validation via dissipation of isothermal pressure
waves" initialises rho = rho0 + drho sin(2 pi x / Nx) at a uniform velocity
U0).  Every field here is sampled at integer node positions x, y, z.

Layout: ``rho`` has numpy shape ``(ny, nx)`` (2-D) or ``(nz, ny, nx)`` (3-D),
x fastest; ``u`` has shape ``(D, *rho.shape)``.  All arrays are float64.
"""
from __future__ import annotations

import math

import numpy as np


def _axes2(nx: int, ny: int):
    y, x = np.meshgrid(np.arange(ny, dtype=np.float64), np.arange(nx, dtype=np.float64),
                       indexing="ij")
    return x, y


def _axes3(nx: int, ny: int, nz: int):
    z, y, x = np.meshgrid(np.arange(nz, dtype=np.float64), np.arange(ny, dtype=np.float64),
                          np.arange(nx, dtype=np.float64), indexing="ij")
    return x, y, z


def taylor_green_2d(n: int, u0: float = 0.05, rho0: float = 1.0, ny: int | None = None):
    """2-D Taylor-Green vortex on an n x ny periodic grid, wavenumber 2 pi / n.

    u_x = -u0 cos(kx) sin(ky), u_y = u0 sin(kx) cos(ky),
    rho = rho0 [1 - (3 u0^2 / 4)(cos 2kx + cos 2ky)] (pressure over c_s^2 = 1/3).
    """
    ny = n if ny is None else ny
    x, y = _axes2(n, ny)
    kx, ky = 2.0 * math.pi / n, 2.0 * math.pi / ny
    ux = -u0 * np.cos(kx * x) * np.sin(ky * y)
    uy = u0 * np.sin(kx * x) * np.cos(ky * y)
    rho = rho0 * (1.0 - 0.75 * u0 * u0 * (np.cos(2 * kx * x) + np.cos(2 * ky * y)))
    return rho, np.stack([ux, uy])


def double_shear_layer(n: int, width: float = 80.0, u0: float = 0.1, delta: float = 0.05):
    """Periodic double shear layer on an n x n grid.

    u_x = u0 tanh((y - n/4) / width) for y <= n/2, u0 tanh((3n/4 - y) / width)
    otherwise; u_y = delta u0 sin(2 pi (x / n + 1/4)) (delta relative to u0);
    rho = 1.
    """
    x, y = _axes2(n, n)
    ux = np.where(y <= n / 2, u0 * np.tanh((y - n / 4) / width), u0 * np.tanh((3 * n / 4 - y) / width))
    uy = delta * u0 * np.sin(2.0 * math.pi * (x / n + 0.25))
    return np.ones((n, n)), np.stack([ux, uy])


def taylor_green_3d(n: int, u0: float = 0.05, rho0: float = 1.0, planes: tuple | None = None):
    """3-D Taylor-Green vortex on an n^3 periodic grid, wavenumber 2 pi / n.

    u_x = u0 sin kx cos ky cos kz, u_y = -u0 cos kx sin ky cos kz, u_z = 0,
    rho = rho0 + (3 rho0 u0^2 / 16)(cos 2kx + cos 2ky)(cos 2kz + 2).
    planes = (z0, z1): only the planes z0 <= z < z1 (a z-slab of the field).
    """
    z0, z1 = (0, n) if planes is None else planes
    z, y, x = np.meshgrid(np.arange(z0, z1, dtype=np.float64), np.arange(n, dtype=np.float64),
                          np.arange(n, dtype=np.float64), indexing="ij")
    k = 2.0 * math.pi / n
    ux = u0 * np.sin(k * x) * np.cos(k * y) * np.cos(k * z)
    uy = -u0 * np.cos(k * x) * np.sin(k * y) * np.cos(k * z)
    uz = np.zeros_like(ux)
    rho = rho0 + (3.0 * rho0 * u0 * u0 / 16.0) * (np.cos(2 * k * x) + np.cos(2 * k * y)) * (np.cos(2 * k * z) + 2.0)
    return rho, np.stack([ux, uy, uz])


def taylor_green_3d_box(nx: int, ny: int, nz: int, u0: float = 0.05, rho0: float = 1.0):
    """The 3-D Taylor-Green field of taylor_green_3d on an nx x ny x nz box, with
    one wavelength per axis (k_a = 2 pi / n_a):

    u_x = u0 sin kx x cos ky y cos kz z, u_y = -u0 cos kx x sin ky y cos kz z, u_z = 0,
    rho = rho0 + (3 rho0 u0^2 / 16)(cos 2kx x + cos 2ky y)(cos 2kz z + 2).
    """
    x, y, z = _axes3(nx, ny, nz)
    kx, ky, kz = 2.0 * math.pi / nx, 2.0 * math.pi / ny, 2.0 * math.pi / nz
    ux = u0 * np.sin(kx * x) * np.cos(ky * y) * np.cos(kz * z)
    uy = -u0 * np.cos(kx * x) * np.sin(ky * y) * np.cos(kz * z)
    rho = rho0 + (3.0 * rho0 * u0 * u0 / 16.0) * (np.cos(2 * kx * x) + np.cos(2 * ky * y)) * (np.cos(2 * kz * z) + 2.0)
    return rho, np.stack([ux, uy, np.zeros_like(ux)])


def shear_wave(nx: int, ny: int, amp: float, rho0: float = 1.0, nz: int | None = None):
    """Transverse shear wave u_x = amp sin(2 pi y / ny), other components 0, rho = rho0.

    2-D when nz is None, else 3-D with the same profile in every z plane.
    """
    if nz is None:
        x, y = _axes2(nx, ny)
        ux = amp * np.sin(2.0 * math.pi * y / ny)
        return np.full((ny, nx), rho0), np.stack([ux, np.zeros_like(ux)])
    x, y, z = _axes3(nx, ny, nz)
    ux = amp * np.sin(2.0 * math.pi * y / ny)
    return np.full((nz, ny, nx), rho0), np.stack([ux, np.zeros_like(ux), np.zeros_like(ux)])


def pressure_wave(nx: int, drho: float, U0: float, rho0: float = 1.0, ny: int = 1, nz: int | None = None):
    """Isothermal pressure wave rho = rho0 + drho sin(2 pi x / nx) carried at a
    uniform velocity U0 along x.  1-D when ny == 1 and nz is None (shape (nx,)),
    2-D (ny, nx) when nz is None, else 3-D (nz, ny, nx)."""
    if nz is None and ny == 1:
        x = np.arange(nx, dtype=np.float64)
        rho = rho0 + drho * np.sin(2.0 * math.pi * x / nx)
        return rho, np.full((1, nx), U0)
    if nz is None:
        x, _ = _axes2(nx, ny)
        rho = rho0 + drho * np.sin(2.0 * math.pi * x / nx)
        return rho, np.stack([np.full_like(rho, U0), np.zeros_like(rho)])
    x, _, _ = _axes3(nx, ny, nz)
    rho = rho0 + drho * np.sin(2.0 * math.pi * x / nx)
    return rho, np.stack([np.full_like(rho, U0), np.zeros_like(rho), np.zeros_like(rho)])


def random_field(shape, seed: int, umax: float = 0.3, rho_lo: float = 0.8, rho_hi: float = 1.2):
    """Node-wise independent random state: rho ~ U[rho_lo, rho_hi], each u_alpha ~
    U(-umax, umax).  A rough field that exercises every population of every node."""
    rng = np.random.default_rng(seed)
    D = len(shape)
    rho = rng.uniform(rho_lo, rho_hi, size=shape)
    u = rng.uniform(-umax, umax, size=(D,) + tuple(shape))
    return rho, u


def batch_domains(count: int = 512, seed: int = 2303, lo: int = 32, hi: int = 512):
    """Parameters of the batched shear-wave workload: `count` independent D2Q9
    domains with nx, ny uniform integers in [lo, hi], wave amplitude
    a ~ U[0.01, 0.2] and viscosity nu log-uniform in [1e-5, 1e-1]
    (tau = 1/2 + 3 nu in lattice units)."""
    rng = np.random.default_rng(seed)
    nx = rng.integers(lo, hi + 1, size=count)
    ny = rng.integers(lo, hi + 1, size=count)
    amp = rng.uniform(0.01, 0.2, size=count)
    nu = np.exp(rng.uniform(math.log(1e-5), math.log(1e-1), size=count))
    return [dict(nx=int(nx[i]), ny=int(ny[i]), amp=float(amp[i]), nu=float(nu[i]),
                 tau=0.5 + 3.0 * float(nu[i])) for i in range(count)]


def serving_trace(n_requests: int = 1000, rate: float = 200.0, seed: int = 8163,
                  d2_range=(64, 1024), d3_range=(32, 192), steps_range=(200, 5000)):
    """Poisson request stream of mixed simulations.

    Arrivals: exponential gaps with mean 1 / rate seconds.  Each request is
    D2Q9 (square, side log-uniform in d2_range) or D3Q27 (cube, side
    log-uniform in d3_range) with probability 1/2; initial field Taylor-Green or
    shear wave with probability 1/2; u0 ~ U[0.01, 0.15]; tau ~ U[0.5001, 0.6];
    steps uniform integer in steps_range.
    """
    rng = np.random.default_rng(seed)
    t = 0.0
    out = []
    for i in range(n_requests):
        t += rng.exponential(1.0 / rate)
        three_d = bool(rng.random() < 0.5)
        lo, hi = d3_range if three_d else d2_range
        side = int(round(math.exp(rng.uniform(math.log(lo), math.log(hi)))))
        out.append(dict(id=i, arrival=t, lattice=27 if three_d else 9, n=side,
                        init="taylor_green" if rng.random() < 0.5 else "shear_wave",
                        u0=float(rng.uniform(0.01, 0.15)), tau=float(rng.uniform(0.5001, 0.6)),
                        steps=int(rng.integers(steps_range[0], steps_range[1] + 1))))
    return out


def request_fields(req: dict):
    """Initial (rho, u) of a serving request."""
    n = req["n"]
    if req["lattice"] == 9:
        if req["init"] == "taylor_green":
            return taylor_green_2d(n, req["u0"])
        return shear_wave(n, n, req["u0"])
    if req["init"] == "taylor_green":
        return taylor_green_3d(n, req["u0"])
    return shear_wave(n, n, req["u0"], nz=n)
