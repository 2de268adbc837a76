"""Plain FP64 CPU oracle of the von Neumann linear-stability analysis
(arXiv:2303.08163, Sec. "Linear stability analysis").

TEST INFRASTRUCTURE ONLY, like the rest of ``oracle/``: only ``tests/``,
``__graft_entry__.smoke()`` and the CPU-baseline leg of ``bench.py`` use it.

Following Sec. "von Neumann spectral analysis: introduction": a plane-wave
perturbation f'_i = F_i exp(i (k . r - omega t)) of the state
f = f^eq(rho, u) evolves by eq. (PerturbedDiscreteLBE); with
E_ij = exp(-i c_i . k) delta_ij the amplification matrix is
M = E (I + J) (eq. VN_eigen), J the collision Jacobian
(``oracle.jacobian``), and each eigenvalue is lambda = exp(-i omega).
Hence, per step, a mode is damped by -ln|lambda| and travels at
-arg(lambda) / |k| along k.

The eigenvalues come from LAPACK's general complex eigensolver
(``numpy.linalg.eigvals``), a library primitive used as one step.

Stability domain (Sec. "Linear stability domain"): a state is linearly
stable when no mode grows, i.e. every |lambda| <= 1, for all wave vectors
k = (k_x, k_y) in [0, pi]^2 and velocity directions theta in [0, pi/2]
(u = |u| (cos theta, sin theta)); here ``tol`` absorbs rounding in the
eigenvalues (|lambda| <= 1 + tol).  The largest stable speed along a
direction is found by bisection, reading the stable set as an interval
[0, u_max) in |u| (the figures of the paper show it so).
"""
from __future__ import annotations

import math

import numpy as np

from . import jacobian, lattice

NU_OF_TAU = 1.0 / 3.0  # nu = varsigma^2 (tau - 1/2)


def tau_of_nu(nu: float) -> float:
    return 0.5 + nu / NU_OF_TAU


def amplification_matrix(tau: float, u, k, corr="off", kind: str = "entropic") -> np.ndarray:
    """M = E (I + J) of eq. (VN_eigen) at the uniform state (rho = 1, u) and
    wave vector k (both of length D), in the oracle's population order."""
    u = np.asarray(u, dtype=np.float64)
    k = np.asarray(k, dtype=np.float64)
    D = u.shape[0]
    c, _ = lattice(D)
    J = jacobian(tau, u, corr=corr, kind=kind)
    E = np.exp(-1j * (c @ k))
    return E[:, None] * (np.eye(len(E)) + J)


def eigenvalues(tau: float, u, k, corr="off", kind: str = "entropic") -> np.ndarray:
    return np.linalg.eigvals(amplification_matrix(tau, u, k, corr, kind))


def spectral_radius(tau: float, u, k, corr="off", kind: str = "entropic") -> float:
    return float(np.max(np.abs(eigenvalues(tau, u, k, corr, kind))))


def batch_spectral_radius(tau: float, u, ks, corr="off", kind: str = "entropic") -> np.ndarray:
    """Spectral radius of M for one state and many wave vectors ks (n, D)."""
    u = np.asarray(u, dtype=np.float64)
    ks = np.asarray(ks, dtype=np.float64)
    D = u.shape[0]
    c, _ = lattice(D)
    J = jacobian(tau, u, corr=corr, kind=kind)
    E = np.exp(-1j * (ks @ c.T))  # (n, Q)
    M = E[:, :, None] * (np.eye(c.shape[0]) + J)[None, :, :]
    return np.max(np.abs(np.linalg.eigvals(M)), axis=1)


def k_grid(n: int = 33, D: int = 2) -> np.ndarray:
    """n points per axis on [0, pi], both ends included; shape (n^D, D)."""
    ax = np.linspace(0.0, math.pi, n)
    if D == 1:
        return ax[:, None]
    kx, ky = np.meshgrid(ax, ax, indexing="ij")
    return np.stack([kx.ravel(), ky.ravel()], axis=1)


def velocity(speed: float, theta: float) -> np.ndarray:
    return np.array([speed * math.cos(theta), speed * math.sin(theta)])


def stable(tau: float, u, ks, corr="off", kind: str = "entropic", tol: float = 1e-9) -> bool:
    u = np.asarray(u, dtype=np.float64)
    if np.any(np.abs(u) >= 1.0):
        return False  # outside the entropic equilibrium's domain
    return bool(np.max(batch_spectral_radius(tau, u, ks, corr, kind)) <= 1.0 + tol)


def max_stable_speed(nu: float, theta: float, ks, corr="off", kind: str = "entropic",
                     tol: float = 1e-9, iters: int = 30) -> float:
    """Largest |u| along direction theta with every mode stable (bisection on
    [0, s_max), s_max the edge of |u_a| < 1 along theta)."""
    tau = tau_of_nu(nu)
    s_max = 1.0 / max(abs(math.cos(theta)), abs(math.sin(theta)))
    lo, hi = 0.0, s_max
    if not stable(tau, velocity(0.0, theta), ks, corr, kind, tol):
        return 0.0
    for _ in range(iters):
        mid = 0.5 * (lo + hi)
        if stable(tau, velocity(mid, theta), ks, corr, kind, tol):
            lo = mid
        else:
            hi = mid
    return lo


def acoustic_modes(tau: float, u: float, k: float, corr="off", kind: str = "entropic"):
    """1-D (D1Q3) acoustic pair at small k along x: returns [(speed, damping)]
    for the two modes whose eigenvalues lie closest to 1, speed = -arg(lambda)/k,
    damping = -ln|lambda| / k^2 (the dissipation coefficient)."""
    lam = eigenvalues(tau, [u], [k], corr, kind)
    lam = lam[np.argsort(np.abs(lam - 1.0))][:2]
    out = [(-np.angle(x) / k, -math.log(abs(x)) / (k * k)) for x in lam]
    return sorted(out)
