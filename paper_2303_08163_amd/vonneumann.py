"""Linear (von Neumann) stability analysis on the GPU (Sec. "Linear stability
analysis" of arXiv:2303.08163).

spectra():           eigenvalues of the amplification matrix M = E (I + J) for
                     a batch of (tau, u, k) cases (lbm_vn_spectra).
max_radius():        largest spectral radius over the [0, pi]^2 wave-vector grid
                     for a batch of states (lbm_vn_max_radius).
stability_domain():  largest stable speed |u| per (nu, theta), theta the angle
                     of u from the x axis, found by bisection run for every
                     (nu, theta) pair at once: each bisection step is one
                     lbm_vn_max_radius call over all pairs (Sec. "Linear
                     stability domain": stable when no mode grows for any k in
                     [0, pi]^2; here |lambda| <= 1 + tol, tol absorbing
                     rounding).  The stable set along a direction is read as
                     the interval [0, u_max).
stability_domains(): the same for several equilibria in lockstep: each
                     bisection step enqueues one call per equilibrium and
                     waits once, so the host's round trip between steps is
                     paid once per step, not once per call.
Every matrix and eigenvalue is computed in the library's kernels; the host
only forms the inputs and keeps the bisection brackets.
"""
from __future__ import annotations

import math

import numpy as np

from . import lbm

NU_PER_TAU = 1.0 / 3.0


def tau_of_nu(nu: float) -> float:
    return 0.5 + nu / NU_PER_TAU


def _lattice(dim: int) -> int:
    if dim == 1:
        return lbm.LBM_D1Q3
    if dim == 2:
        return lbm.LBM_D2Q9
    raise ValueError("von Neumann spectra run on D1Q3 or D2Q9")


def spectra(cases, dim: int = 2, equilibrium="entropic", bulk_correction=False, device="cuda:0"):
    """cases (n, 5): tau, u_x, u_y, k_x, k_y.  Returns (radius (n,), eigenvalues
    (n, Q) complex, info (n,) QR steps or -1) as numpy arrays."""
    import torch
    lbm.load_library()
    c = torch.as_tensor(np.ascontiguousarray(cases, dtype=np.float64)).to(device)
    n = c.shape[0]
    if c.ndim != 2 or c.shape[1] != 5:
        raise ValueError("cases must have shape (n, 5)")
    Q = 3 ** dim
    radius = torch.empty(n, dtype=torch.float64, device=device)
    eig = torch.empty((n, Q, 2), dtype=torch.float64, device=device)
    info = torch.empty(n, dtype=torch.int32, device=device)
    stream = torch.cuda.current_stream(device)
    lbm.lbm_vn_spectra(_lattice(dim), equilibrium, bulk_correction, c.data_ptr(), n, radius.data_ptr(),
                       eig.data_ptr(), info.data_ptr(), None, stream.cuda_stream)
    stream.synchronize()
    e = eig.cpu().numpy()
    return radius.cpu().numpy(), e[..., 0] + 1j * e[..., 1], info.cpu().numpy()


class RadiusEvaluator:
    """Device buffers for repeated lbm_vn_max_radius calls over up to n_states states."""

    def __init__(self, n_states: int, dim: int = 2, equilibrium="entropic", bulk_correction=False, nk: int = 33,
                 device="cuda:0"):
        import torch
        lbm.load_library()
        self.dim, self.eq, self.corr, self.nk = dim, equilibrium, bulk_correction, nk
        self.device = torch.device(device)
        self.capacity = n_states
        # pinned staging, so that enqueueing a call does not wait for the stream
        self.host_states = torch.empty((n_states, 3), dtype=torch.float64, pin_memory=True)
        self.states = torch.empty((n_states, 3), dtype=torch.float64, device=self.device)
        self.rmax = torch.empty(n_states, dtype=torch.float64, device=self.device)
        self.scratch = torch.empty(n_states, dtype=torch.int64, device=self.device)
        self.unconverged = torch.zeros(1, dtype=torch.int32, device=self.device)
        # a stream of its own (default priority): the calls of evaluators run in
        # lockstep overlap on the GPU, one kernel's last wavefronts beside the
        # next one's first
        self.stream = torch.cuda.Stream(device=self.device)
        for t in (self.states, self.rmax, self.scratch, self.unconverged):
            t.record_stream(self.stream)  # not reused before that stream's work is done
        self.matrices = 0
        self.n = 0

    def launch(self, states: np.ndarray) -> None:
        """Enqueue one call over states (n, 3): tau, u_x, u_y (no wait).  The
        staging buffer is reused, so result() must come before the next launch."""
        import torch
        n = states.shape[0]
        if n > self.capacity:
            raise ValueError("more states than the evaluator holds")
        self.host_states[:n].numpy()[:] = states
        with torch.cuda.stream(self.stream):
            self.states[:n].copy_(self.host_states[:n], non_blocking=True)
        lbm.lbm_vn_max_radius(_lattice(self.dim), self.eq, self.corr, self.states.data_ptr(), n, self.nk,
                              self.rmax.data_ptr(), self.scratch.data_ptr(), self.unconverged.data_ptr(),
                              self.stream.cuda_stream)
        self.matrices += n * self.nk ** self.dim
        self.n = n

    def result(self):
        """(max radius (n,), unconverged count) of the last launch; waits for it."""
        import torch
        with torch.cuda.stream(self.stream):
            r = self.rmax[:self.n].cpu().numpy()  # waits for the evaluator's stream
            bad = int(self.unconverged.item())
        return r, bad

    def __call__(self, states: np.ndarray):
        """states (n, 3): tau, u_x, u_y.  Returns (max radius (n,), unconverged count)."""
        self.launch(np.asarray(states, dtype=np.float64))
        return self.result()


def max_radius(states, dim: int = 2, equilibrium="entropic", bulk_correction=False, nk: int = 33,
               device="cuda:0"):
    states = np.asarray(states, dtype=np.float64)
    ev = RadiusEvaluator(states.shape[0], dim, equilibrium, bulk_correction, nk, device)
    return ev(states)


def stability_domains(nus, thetas, equilibria=("entropic", "poly2", "product"), bulk_correction=False,
                      nk: int = 33, iters: int = 24, tol: float = 1e-9, device="cuda:0"):
    """Largest stable speed for every (nu, theta) pair and every equilibrium;
    returns {equilibrium: (u_max array of shape (len(nus), len(thetas)), stats
    dict)}.  The bisections run in lockstep (one wait per step for all
    equilibria); each equilibrium's calls and results are those of
    stability_domain alone."""
    nus = np.asarray(nus, dtype=np.float64)
    thetas = np.asarray(thetas, dtype=np.float64)
    P = len(nus) * len(thetas)
    nu_p = np.repeat(nus, len(thetas))
    th_p = np.tile(thetas, len(nus))
    tau_p = 0.5 + nu_p / NU_PER_TAU
    cos_p, sin_p = np.cos(th_p), np.sin(th_p)
    s_max = 1.0 / np.maximum(np.abs(cos_p), np.abs(sin_p))
    evs = {eq: RadiusEvaluator(P, 2, eq, bulk_correction, nk, device) for eq in equilibria}
    unconverged = {eq: 0 for eq in equilibria}

    def stable(speeds):
        for eq, ev in evs.items():
            ev.launch(np.stack([tau_p, speeds[eq] * cos_p, speeds[eq] * sin_p], axis=1))
        out = {}
        for eq, ev in evs.items():
            r, bad = ev.result()
            unconverged[eq] += bad
            out[eq] = r <= 1.0 + tol
        return out

    lo = {eq: np.zeros(P) for eq in equilibria}
    hi = {eq: s_max.copy() for eq in equilibria}
    ok0 = stable({eq: np.zeros(P) for eq in equilibria})
    for _ in range(iters):
        mid = {eq: 0.5 * (lo[eq] + hi[eq]) for eq in equilibria}
        s = stable(mid)
        for eq in equilibria:
            lo[eq] = np.where(s[eq], mid[eq], lo[eq])
            hi[eq] = np.where(s[eq], hi[eq], mid[eq])
    return {eq: (np.where(ok0[eq], lo[eq], 0.0).reshape(len(nus), len(thetas)),
                 {"matrices": evs[eq].matrices, "unconverged": unconverged[eq], "calls": iters + 1})
            for eq in equilibria}


def stability_domain(nus, thetas, equilibrium="entropic", bulk_correction=False, nk: int = 33, iters: int = 24,
                     tol: float = 1e-9, device="cuda:0"):
    """Largest stable speed for every (nu, theta) pair; returns (u_max array of
    shape (len(nus), len(thetas)), stats dict)."""
    return stability_domains(nus, thetas, (equilibrium,), bulk_correction, nk, iters, tol, device)[equilibrium]


PAPER_NUS = [1e-6, 5e-6, 1e-5, 5e-5, 1e-4, 5e-4, 1e-3, 5e-3, 1e-2, 5e-2, 0.1, 0.5, 1.0, 1.1, 1.2]
