"""Pins of the oracle's lattice and equilibria against facts fixed by the paper and
by mathematics, not by re-typing the oracle's formulas:

* lattice: the 1-D weights {1/6, 2/3, 1/6} and their tensor products
  (Sec. "Basic concepts"), isotropy of the second moment with varsigma^2 = 1/3;
* entropic equilibrium (eq. Entropic_isothermal_EDF): the mass and momentum
  constraints it is defined by (Sec. "Discrete entropic equilibrium
  construction"), the rest state, a brute-force minimisation of
  H = sum f ln(f / w) under those constraints, H-minimality under
  moment-preserving perturbations, the pressure deviation P* printed in
  Sec. "Conservation equations", and a high-precision evaluation of an
  algebraically equivalent product of 1-D factors;
* polynomial and product-form equilibria (Sec. "Polynomial discrete
  equilibria"): their defining moments, and the low-Mach agreement of the
  entropic equilibrium with them (orders u^3 and u^4).
"""
import itertools

import mpmath
import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0


@pytest.mark.parametrize("D", [1, 2, 3])
def test_lattice_is_tensor_product_of_1d(D):
    c, w = oracle.lattice(D)
    Q = 3 ** D
    assert c.shape == (Q, D) and w.shape == (Q,)
    assert sorted(map(tuple, c)) == sorted(itertools.product((-1, 0, 1), repeat=D))
    w1 = {-1: 1 / 6, 0: 2 / 3, 1: 1 / 6}
    for ci, wi in zip(c, w):
        assert wi == pytest.approx(np.prod([w1[int(a)] for a in ci]), rel=1e-15)
    assert np.sum(w) == pytest.approx(1.0, abs=1e-15)
    assert np.allclose(w @ c, 0.0, atol=1e-16)
    # second-moment isotropy: sum w c_a c_b = varsigma^2 delta_ab with varsigma^2 = 1/3
    assert np.allclose(np.einsum("i,ia,ib->ab", w, c, c), CS2 * np.eye(D), atol=1e-15)


def test_d3q27_weight_values():
    _, w = oracle.lattice(3)
    assert sorted(set(np.round(w * 216).astype(int))) == [1, 4, 16, 64]  # 1/216, 1/54, 2/27, 8/27
    assert np.isclose(np.max(w), 8 / 27) and np.isclose(np.min(w), 1 / 216)


def _random_states(D, n, seed, umax=0.95):
    rng = np.random.default_rng(seed)
    return [(rng.uniform(0.2, 3.0), rng.uniform(-umax, umax, D)) for _ in range(n)]


def _cond(u):
    """Rounding amplification of the closed form: X^{-1} holds the factors
    2 - S_a with S_a = sqrt(1 + 3 u_a^2), whose relative rounding error is about
    eps S / (2 - S), large as |u_a| -> 1."""
    S = np.sqrt(1 + 3 * np.asarray(u) ** 2)
    return float(np.sum(2.0 + 2.0 * S / (2.0 - S)))


@pytest.mark.parametrize("D", [1, 2, 3])
def test_entropic_conserves_mass_and_momentum(D):
    c, _ = oracle.lattice(D)
    for rho, u in _random_states(D, 200, seed=10 + D):
        f, bad = oracle.equilibrium(rho, u)
        assert not bad
        assert np.all(f > 0)
        tol = 2.2e-16 * (D + 4 + _cond(u)) * rho
        assert abs(f.sum() - rho) <= tol
        assert np.max(np.abs(c.T @ f - rho * u)) <= 2 * tol


@pytest.mark.parametrize("D", [1, 2, 3])
def test_entropic_rest_state_is_weights(D):
    _, w = oracle.lattice(D)
    f, _ = oracle.equilibrium(1.7, np.zeros(D))
    assert np.allclose(f, 1.7 * w, rtol=2e-16, atol=0)


def _newton_dual(D, rho, u, iters=60):
    """Minimise H = sum f ln(f/w) subject to sum f = rho, sum c f = rho u by
    Newton on the convex dual: f_i = w_i exp(lam . phi_i), phi_i = (1, c_i)."""
    c, w = oracle.lattice(D)
    phi = np.hstack([np.ones((len(w), 1)), c.astype(float)])
    m = np.concatenate([[rho], rho * np.asarray(u)])
    lam = np.zeros(D + 1)
    lam[0] = np.log(rho)
    for _ in range(iters):
        f = w * np.exp(phi @ lam)
        g = phi.T @ f - m
        H = (phi * f[:, None]).T @ phi
        step = np.linalg.solve(H, g)
        lam -= step
        if np.max(np.abs(step)) < 1e-16:
            break
    return w * np.exp(phi @ lam)


@pytest.mark.parametrize("D", [1, 2, 3])
def test_entropic_equals_brute_force_entropy_minimiser(D):
    for rho, u in _random_states(D, 40, seed=20 + D, umax=0.9):
        f_ref = _newton_dual(D, rho, u)
        f, _ = oracle.equilibrium(rho, u)
        assert np.max(np.abs(f - f_ref) / f_ref) < 1e-13 * _cond(u)


def test_entropic_equals_minimiser_high_precision():
    """Newton on the dual in 40-digit arithmetic at two D2Q9 states."""
    mpmath.mp.dps = 40
    c, w = oracle.lattice(2)
    for rho, u in [(1.1, (0.1, -0.2)), (0.7, (0.85, 0.6))]:
        rho_m = mpmath.mpf(rho)
        u_m = [mpmath.mpf(x) for x in u]
        wm = [mpmath.mpf(1) / 6, mpmath.mpf(2) / 3, mpmath.mpf(1) / 6]
        wq = [wm[int(ci[0]) + 1] * wm[int(ci[1]) + 1] for ci in c]
        lam = [mpmath.log(rho_m), mpmath.mpf(0), mpmath.mpf(0)]
        for _ in range(80):
            f = [wq[i] * mpmath.exp(lam[0] + lam[1] * int(c[i][0]) + lam[2] * int(c[i][1]))
                 for i in range(9)]
            phi = [[1, int(ci[0]), int(ci[1])] for ci in c]
            m = [rho_m, rho_m * u_m[0], rho_m * u_m[1]]
            g = mpmath.matrix([sum(phi[i][a] * f[i] for i in range(9)) - m[a] for a in range(3)])
            H = mpmath.matrix(3, 3)
            for a in range(3):
                for b in range(3):
                    H[a, b] = sum(phi[i][a] * phi[i][b] * f[i] for i in range(9))
            step = mpmath.lu_solve(H, g)
            lam = [lam[a] - step[a] for a in range(3)]
        f_ref = np.array([float(x) for x in f])
        f_or, _ = oracle.equilibrium(rho, np.array(u))
        assert np.max(np.abs(f_or - f_ref) / f_ref) < 2e-15


@pytest.mark.parametrize("D", [2, 3])
def test_entropic_minimises_H_under_moment_preserving_perturbations(D):
    c, w = oracle.lattice(D)
    rng = np.random.default_rng(30 + D)
    phi = np.hstack([np.ones((len(w), 1)), c.astype(float)])
    # basis of perturbations that keep mass and momentum: null space of phi^T
    _, _, vt = np.linalg.svd(phi.T)
    null = vt[D + 1:]
    for rho, u in _random_states(D, 20, seed=40 + D, umax=0.8):
        f, _ = oracle.equilibrium(rho, u)
        H0 = np.sum(f * np.log(f / w))
        for _ in range(50):
            d = rng.standard_normal(null.shape[0]) @ null
            d *= 1e-3 * np.min(f) / np.max(np.abs(d))
            g = f + d
            assert np.allclose(phi.T @ d, 0, atol=1e-15)
            assert np.sum(g * np.log(g / w)) > H0


def test_entropic_product_of_1d_factors_high_precision():
    """The entropic equilibrium factorises as rho prod_alpha g_{c_alpha}(u_alpha) with
    S = sqrt(1 + 3u^2), g_0 = 2(2 - S)/3, g_{+-1} = (2S - 1 +- 3u)/6 (an algebraic
    rearrangement of Z and X^{-1}).  Evaluated in 40 digits, it pins the oracle's
    use of Z_alpha^{c} (sign of c, which factor divides) at every population."""
    mpmath.mp.dps = 40
    for D in (1, 2, 3):
        c, _ = oracle.lattice(D)
        for rho, u in _random_states(D, 30, seed=50 + D, umax=0.97):
            g = []
            for a in range(D):
                ua = mpmath.mpf(float(u[a]))
                S = mpmath.sqrt(1 + 3 * ua * ua)
                g.append({-1: (2 * S - 1 - 3 * ua) / 6, 0: 2 * (2 - S) / 3, 1: (2 * S - 1 + 3 * ua) / 6})
            ref = np.array([float(mpmath.mpf(float(rho)) * mpmath.fprod(g[a][int(ci[a])] for a in range(D)))
                            for ci in c])
            f, _ = oracle.equilibrium(rho, u)
            assert np.max(np.abs(f - ref) / ref) < 2.2e-16 * (3 * D + 4 + 2 * _cond(u))


@pytest.mark.parametrize("D", [1, 2, 3])
def test_entropic_pressure_deviation_matches_paper(D):
    """P*_aa = sum (c_a - u_a)^2 f^eq - rho varsigma^2 equals the closed form
    -rho varsigma^2 [(u_a/varsigma)^2 - 2 sqrt((u_a/varsigma)^2 + 1) + 2]
    given in Sec. "Conservation equations"."""
    c, _ = oracle.lattice(D)
    for rho, u in _random_states(D, 100, seed=60 + D):
        f, _ = oracle.equilibrium(rho, u)
        for a in range(D):
            pstar = np.sum((c[:, a] - u[a]) ** 2 * f) - rho * CS2
            v2 = u[a] ** 2 / CS2
            closed = -rho * CS2 * (v2 - 2 * np.sqrt(v2 + 1) + 2)
            assert abs(pstar - closed) < 2.2e-16 * (8 + 2 * _cond(u)) * rho


@pytest.mark.parametrize("D", [1, 2, 3])
def test_polynomial_equilibria_moments(D):
    """poly2 matches the Maxwell-Boltzmann moments up to second order; the
    product form matches mass, momentum and the diagonal second moments
    rho (varsigma^2 + u_a^2) (Sec. "Polynomial discrete equilibria"; both have
    P* = 0, Sec. "Conservation equations")."""
    c, _ = oracle.lattice(D)
    for rho, u in _random_states(D, 50, seed=70 + D, umax=0.4):
        for kind in ("poly2", "product"):
            f, _ = oracle.equilibrium(rho, u, kind=kind)
            assert abs(f.sum() - rho) < 1e-14 * rho
            assert np.allclose(c.T @ f, rho * u, atol=1e-14 * rho)
            P = np.einsum("i,ia,ib->ab", f, c, c)
            assert np.allclose(np.diag(P), rho * (CS2 + u ** 2), atol=1e-14 * rho)
            if kind == "poly2":
                assert np.allclose(P, rho * (CS2 * np.eye(D) + np.outer(u, u)), atol=1e-14 * rho)


@pytest.mark.parametrize("D", [2, 3])
def test_low_mach_orders(D):
    """Entropic minus poly2 is O(u^3), entropic minus product form is O(u^4):
    halving |u| divides the max deviation by 8 and 16."""
    rng = np.random.default_rng(80 + D)
    for _ in range(5):
        direction = rng.standard_normal(D)
        direction /= np.linalg.norm(direction)
        errs = {"poly2": [], "product": []}
        for s in (0.04, 0.02, 0.01):
            u = s * direction
            fe, _ = oracle.equilibrium(1.0, u)
            for kind in errs:
                fk, _ = oracle.equilibrium(1.0, u, kind=kind)
                errs[kind].append(np.max(np.abs(fe - fk)))
        for kind, order in (("poly2", 8.0), ("product", 16.0)):
            r = np.array(errs[kind][:-1]) / np.array(errs[kind][1:])
            assert np.all(np.abs(r / order - 1) < 0.1), (kind, r)


def test_domain_flag():
    assert oracle.equilibrium(1.0, np.array([0.999, 0.0]))[1] is False
    assert oracle.equilibrium(1.0, np.array([1.0, 0.0]))[1] is True
    assert oracle.equilibrium(1.0, np.array([0.0, -1.2]))[1] is True
    assert oracle.equilibrium(0.0, np.array([0.0, 0.0]))[1] is True
    assert oracle.equilibrium(float("nan"), np.array([0.0, 0.0]))[1] is True
