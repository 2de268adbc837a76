"""GPU parity of the von Neumann spectra (lbm_vn_spectra, lbm_vn_max_radius)
against the oracle (oracle.stability: the same amplification matrix built
from oracle.jacobian, eigenvalues from LAPACK).

Eigenvalues are unordered, so they are compared as multisets (greedy nearest
matching) and through the unique spectral radius.  Tolerance: a backward-stable
eigensolver returns the eigenvalues of M + dM with |dM| ~ c eps |M|, and by the
Bauer-Fike theorem an eigenvalue moves by at most kappa(V) |dM|, kappa(V) the
condition number of the eigenvector matrix.  Both sides are backward stable, so
the bound used is 1e-13 kappa(V) |M|_2 (c ~ 450).

Stability-domain searches are compared with the oracle's bisection run with the
same grid, tolerance and step count: the two may differ by one bisection
interval where a spectral radius lies within rounding of 1 + tol.
"""
import math

import numpy as np
import pytest

from oracle import stability as ost

pytestmark = pytest.mark.gpu

KINDS = ["entropic", "poly2", "product"]
CS = 1.0 / math.sqrt(3.0)


def _vn():
    from paper_2303_08163_amd import vonneumann
    return vonneumann


def random_cases(D, n, seed):
    rng = np.random.default_rng(seed)
    tau = 0.5 + 3 * np.exp(rng.uniform(np.log(1e-6), np.log(1.2), n))
    if D == 1:
        ux, uy = rng.uniform(-0.95, 0.95, n), np.zeros(n)
    else:
        sp, th = rng.uniform(0, 0.95, n), rng.uniform(0, np.pi / 2, n)
        ux, uy = sp * np.cos(th), sp * np.sin(th)
    kx, ky = rng.uniform(0, np.pi, n), rng.uniform(0, np.pi, n)
    kx[:5], ky[:5] = [0, np.pi, 1e-4, 0, np.pi], [0, np.pi, 0, 1e-4, 0]
    tau[5] = 1.0  # omega = 1: six zero eigenvalues
    return np.stack([tau, ux, uy, kx, ky], axis=1)


@pytest.mark.parametrize("D", [1, 2])
@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("corr", [False, True])
def test_spectra_match_lapack(D, kind, corr):
    vn = _vn()
    cases = random_cases(D, 300, seed=10 * D + KINDS.index(kind) + (5 if corr else 0))
    radius, eig, info = vn.spectra(cases, dim=D, equilibrium=kind, bulk_correction=corr)
    assert np.all(info >= 0)
    worst = 0.0
    for t, row in enumerate(cases):
        M = ost.amplification_matrix(row[0], row[1:1 + D], row[3:3 + D], corr="min" if corr else "off", kind=kind)
        ref, V = np.linalg.eig(M)
        bound = 1e-13 * np.linalg.cond(V) * np.linalg.norm(M, 2) + 1e-300
        assert abs(radius[t] - np.max(np.abs(ref))) <= bound, (t, row)
        rem = list(ref)
        for z in eig[t]:
            j = int(np.argmin([abs(z - r) for r in rem]))
            assert abs(z - rem[j]) <= bound, (t, row, z, rem[j])
            rem.pop(j)
        worst = max(worst, abs(radius[t] - np.max(np.abs(ref))) / np.linalg.norm(M, 2))
    print(f"[vn] D{D} {kind} corr={corr}: max |radius - LAPACK| / |M| = {worst:.2e}, "
          f"QR steps mean {info.mean():.1f} max {info.max()}", flush=True)


@pytest.mark.parametrize("D", [1, 2])
def test_spectra_independent_of_wavefront_grouping(D):
    """QR steps sweep the largest active block of any lane of the wavefront, but
    the rows past a lane's own block see only exact identities (zero
    subdiagonals, no shift), so a matrix's eigenvalues and step count do not
    depend on the cases that share its wavefront: a permuted order (1000 cases,
    a ragged last wavefront) and cases run alone (a wavefront of one live lane)
    give bitwise the same results.  Adding 0.0 maps -0 to +0, the one change an
    identity rotation may make."""
    vn = _vn()
    cases = random_cases(D, 1000, seed=77 + D)
    perm = np.random.default_rng(3).permutation(len(cases))
    r1, e1, i1 = vn.spectra(cases, dim=D, equilibrium="product")
    r2, e2, i2 = vn.spectra(cases[perm], dim=D, equilibrium="product")
    assert np.all(i1 >= 0)
    assert np.array_equal(i1[perm], i2)
    assert np.array_equal(r1[perm], r2)
    assert np.array_equal(e1[perm] + 0.0, e2 + 0.0)
    for t in (0, 5, 6, 100, 999, int(np.argmax(i1)), int(np.argmin(i1))):
        ra, ea, ia = vn.spectra(cases[t:t + 1], dim=D, equilibrium="product")
        assert ia[0] == i1[t] and ra[0] == r1[t], t
        assert np.array_equal(ea[0] + 0.0, e1[t] + 0.0), t
    print(f"[vn] D{D}: QR steps per case {i1.min()}..{i1.max()}, grouping-independent", flush=True)


@pytest.mark.parametrize("kind", KINDS)
def test_k0_spectrum(kind):
    vn = _vn()
    cases = np.array([[0.55, 0.3, -0.2, 0.0, 0.0], [2.0, -0.1, 0.6, 0.0, 0.0]])
    _, eig, _ = vn.spectra(cases, equilibrium=kind)
    for row, lam in zip(cases, eig):
        expect = np.sort([1.0 - 1.0 / row[0]] * 6 + [1.0] * 3)
        assert np.max(np.abs(np.sort(lam.real) - expect)) < 1e-12 and np.max(np.abs(lam.imag)) < 1e-12


@pytest.mark.parametrize("u", [-0.8, -0.3, 0.0, 0.45, 0.9])
def test_d1q3_entropic_sound_speeds(u):
    """k -> 0 acoustic phase speeds equal c_s^{e+-} of eqs. (cs_plus_ent), (cs_minus_ent)."""
    vn = _vn()
    k = 1e-3
    _, eig, _ = vn.spectra(np.array([[0.6, u, 0.0, k, 0.0]]), dim=1)
    lam = eig[0][np.argsort(np.abs(eig[0] - 1.0))][:2]
    speeds = np.sort(-np.angle(lam) / k)
    S = math.sqrt((u / CS) ** 2 + 1.0)
    expect = np.sort([(u - CS * math.sqrt(2 * S - 1)) / S, (u + CS * math.sqrt(2 * S - 1)) / S])
    assert np.max(np.abs(speeds - expect)) < 1e-6


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("corr", [False, True])
def test_max_radius_matches_oracle_grid(kind, corr):
    vn = _vn()
    nk = 17
    rng = np.random.default_rng(40 + KINDS.index(kind))
    nus = np.exp(rng.uniform(np.log(1e-6), np.log(1.2), 12))
    sp, th = rng.uniform(0, 0.9, 12), rng.uniform(0, np.pi / 2, 12)
    states = np.stack([0.5 + 3 * nus, sp * np.cos(th), sp * np.sin(th)], axis=1)
    r, bad = vn.max_radius(states, equilibrium=kind, bulk_correction=corr, nk=nk)
    assert bad == 0
    ks = ost.k_grid(nk)
    for s, st in enumerate(states):
        ref = ost.batch_spectral_radius(st[0], st[1:], ks, corr="min" if corr else "off", kind=kind)
        assert abs(r[s] - np.max(ref)) < 1e-10 * max(1.0, np.max(ref)), (s, st)


def test_stability_domain_matches_oracle_bisection():
    vn = _vn()
    nk, iters, tol = 17, 20, 1e-9
    ks = ost.k_grid(nk)
    nus = [1e-5, 0.1]
    thetas = [0.0, math.pi / 8, math.pi / 4]
    for kind in KINDS:
        got, stats = vn.stability_domain(nus, thetas, equilibrium=kind, nk=nk, iters=iters, tol=tol)
        assert stats["unconverged"] == 0
        for a, nu in enumerate(nus):
            for b, th in enumerate(thetas):
                ref = ost.max_stable_speed(nu, th, ks, kind=kind, tol=tol, iters=iters)
                s_max = 1.0 / max(abs(math.cos(th)), abs(math.sin(th)))
                assert abs(got[a, b] - ref) <= s_max * 2.0 ** (1 - iters), (kind, nu, th, got[a, b], ref)


@pytest.mark.parametrize("corr", [False, True])
def test_stability_domains_lockstep_equals_separate(corr):
    """The lockstep sweep over three equilibria (one host wait per bisection
    step) gives each equilibrium exactly the domain, call count and matrix count
    of its own sweep."""
    vn = _vn()
    nus = [1e-6, 1e-3, 0.5]
    thetas = [0.0, math.pi / 8, math.pi / 4, math.pi / 2]
    together = vn.stability_domains(nus, thetas, KINDS, bulk_correction=corr, nk=17, iters=16)
    assert list(together) == KINDS
    for kind in KINDS:
        alone, st = vn.stability_domain(nus, thetas, equilibrium=kind, bulk_correction=corr, nk=17, iters=16)
        got, st_t = together[kind]
        assert np.array_equal(got, alone), kind
        assert st_t == st and st["unconverged"] == 0, (kind, st_t, st)


def test_paper_stability_limits_on_gpu():
    """Sec. "Linear stability domain": polynomial equilibria stop at
    1 - varsigma at large viscosity, the product form reaches 0.598 on the
    diagonal, the entropic equilibrium is stable on the whole lattice."""
    vn = _vn()
    thetas = [0.0, math.pi / 4]
    poly, _ = vn.stability_domain([1.0], thetas, equilibrium="poly2", nk=33, iters=24)
    prod, _ = vn.stability_domain([0.1], thetas, equilibrium="product", nk=33, iters=24)
    ent, _ = vn.stability_domain([1e-6, 1e-5, 0.1, 1.2], thetas, equilibrium="entropic", nk=33, iters=24)
    assert poly[0, 0] == pytest.approx(1.0 - CS, abs=1e-4)
    assert prod[0, 0] == pytest.approx(1.0 - CS, abs=1e-4)
    assert prod[0, 1] == pytest.approx(math.sqrt(2.0) * (1.0 - CS), abs=1e-3)
    s_max = np.array([1.0, math.sqrt(2.0)])
    assert np.all(np.abs(ent - s_max[None, :]) < 1e-5)
