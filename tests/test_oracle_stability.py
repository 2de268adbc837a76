"""Pins of the von Neumann oracle (oracle.jacobian, oracle.stability) against
what the paper and the mathematics fix, not against itself:

  - the Jacobian equals central finite differences of the oracle's own
    equilibrium composed with the moments (a different computation);
  - collision invariants: sum_i J_ij = 0 and sum_i c_ia J_ij = 0;
  - d f^eq / d f = I + J / (2 beta) is a projector (f^eq of an equilibrium is
    itself), so at k = 0 the spectrum of M is 1 (D + 1 times) and 1 - 2 beta;
  - at k -> 0 the two acoustic modes of D1Q3 travel at the sound speeds of
    eqs. (cs_plus_ent), (cs_minus_ent) for the entropic equilibrium and at
    u +- varsigma for the polynomial ones, and their mean dissipation is
    nu A(u) (eq. entropic_bulk / LBGK_bulk), restored to nu by the correction;
  - the shear mode of D2Q9 at rest dissipates at nu k^2;
  - stability limits printed in the paper: the polynomial equilibria reach
    |u| = 1 - varsigma = 0.4226 at large viscosity (eq. CFL_lmit_absolute_poly),
    the product form sqrt(2) (1 - varsigma) = 0.598 along the diagonal, and
    the entropic equilibrium is stable on the whole lattice |u_a| < 1.
"""
import math

import numpy as np
import pytest

import oracle
from oracle import stability as st

CS = 1.0 / math.sqrt(3.0)
KINDS = ["entropic", "poly2", "product"]


def _moments(f, c):
    rho = f.sum()
    return rho, (c.T @ f) / rho


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D,u", [(1, [0.37]), (2, [0.3, -0.45]), (2, [-0.7, 0.05]), (3, [0.2, -0.1, 0.33])])
@pytest.mark.parametrize("corr", ["off", "min"])
def test_jacobian_matches_finite_differences(kind, D, u, corr):
    tau, rho = 0.57, 1.3
    c, _ = oracle.lattice(D)
    feq, _ = oracle.equilibrium(rho, u, kind)
    J = oracle.jacobian(tau, u, corr=corr, kind=kind, rho=rho)
    two_beta = 2.0 * oracle.beta(tau, np.array(u), corr=corr, kind=kind)
    h = 1e-6
    Q = len(feq)
    P = np.zeros((Q, Q))
    for j in range(Q):
        e = np.zeros(Q)
        e[j] = h
        fp, _ = oracle.equilibrium(*_moments(feq + e, c), kind)
        fm, _ = oracle.equilibrium(*_moments(feq - e, c), kind)
        P[:, j] = (fp - fm) / (2 * h)
    assert np.max(np.abs(J - two_beta * (P - np.eye(Q)))) < 1e-8


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D", [1, 2, 3])
def test_jacobian_invariants_and_projector(kind, D):
    rng = np.random.default_rng(D)
    u = rng.uniform(-0.5, 0.5, size=D)
    tau = 0.8
    c, _ = oracle.lattice(D)
    J = oracle.jacobian(tau, u, kind=kind)
    assert np.max(np.abs(J.sum(axis=0))) < 1e-14
    assert np.max(np.abs(c.T @ J)) < 1e-14
    P = np.eye(len(J)) + J * tau  # 2 beta = 1 / tau without the correction
    assert np.max(np.abs(P @ P - P)) < 1e-13


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("D", [1, 2])
def test_k0_spectrum(kind, D):
    tau = 0.55
    u = [0.3, -0.2][:D]
    lam = np.sort(np.real(st.eigenvalues(tau, u, [0.0] * D, kind=kind)))
    Q = 3 ** D
    expect = np.sort([1.0 - 1.0 / tau] * (Q - D - 1) + [1.0] * (D + 1))
    assert np.max(np.abs(lam - expect)) < 1e-12


@pytest.mark.parametrize("u", [-0.9, -0.6, -0.2, 0.0, 0.3, 0.7, 0.9])
def test_entropic_sound_speeds(u):
    S = math.sqrt((u / CS) ** 2 + 1.0)
    c_minus = (u - CS * math.sqrt(2.0 * S - 1.0)) / S
    c_plus = (u + CS * math.sqrt(2.0 * S - 1.0)) / S
    (s1, _), (s2, _) = st.acoustic_modes(0.6, u, 1e-3)
    assert s1 == pytest.approx(c_minus, abs=1e-6) and s2 == pytest.approx(c_plus, abs=1e-6)


@pytest.mark.parametrize("kind", ["poly2", "product"])
@pytest.mark.parametrize("u", [-0.3, 0.0, 0.2, 0.4])
def test_polynomial_sound_speeds(kind, u):
    (s1, _), (s2, _) = st.acoustic_modes(0.6, u, 1e-3, kind=kind)
    assert s1 == pytest.approx(u - CS, abs=1e-6) and s2 == pytest.approx(u + CS, abs=1e-6)


@pytest.mark.parametrize("kind", KINDS)
@pytest.mark.parametrize("u", [-0.35, 0.0, 0.15, 0.3])
def test_mean_acoustic_dissipation_is_nu_A(kind, u):
    tau = 0.6
    nu = (tau - 0.5) / 3.0
    A = oracle.bulk_A(u, "entropic" if kind == "entropic" else "poly2")
    m = st.acoustic_modes(tau, u, 2e-3, kind=kind)
    assert 0.5 * (m[0][1] + m[1][1]) == pytest.approx(nu * A, rel=1e-4)
    mc = st.acoustic_modes(tau, u, 2e-3, corr="min", kind=kind)
    assert 0.5 * (mc[0][1] + mc[1][1]) == pytest.approx(nu, rel=1e-4)


def test_shear_mode_dissipation_at_rest():
    tau, k = 0.7, 2e-3
    nu = (tau - 0.5) / 3.0
    lam = st.eigenvalues(tau, [0.0, 0.0], [0.0, k])
    # the shear mode (u_x varying along y) does not propagate: arg(lambda) ~ 0
    near = lam[np.argsort(np.abs(lam - 1.0))][:3]
    shear = near[np.argmin(np.abs(np.angle(near)))]
    assert -math.log(abs(shear)) / k ** 2 == pytest.approx(nu, rel=1e-4)


@pytest.fixture(scope="module")
def ks():
    return st.k_grid(33)


@pytest.mark.parametrize("kind", ["poly2", "product"])
def test_polynomial_limit_at_large_viscosity(ks, kind):
    s = st.max_stable_speed(1.0, 0.0, ks, kind=kind, iters=24)
    assert s == pytest.approx(1.0 - CS, abs=1e-4)


def test_product_form_diagonal_limit(ks):
    s = st.max_stable_speed(0.1, math.pi / 4, ks, kind="product", iters=24)
    assert s == pytest.approx(math.sqrt(2.0) * (1.0 - CS), abs=1e-3)
    assert s == pytest.approx(0.598, abs=1e-3)


@pytest.mark.parametrize("nu", [1e-6, 1e-5, 0.1, 1.2])
def test_entropic_stable_on_the_whole_lattice(ks, nu):
    tau = st.tau_of_nu(nu)
    for u in ([0.95, 0.0], [0.9, 0.9], [0.5, -0.97], [-0.99, 0.3]):
        assert st.stable(tau, u, ks, kind="entropic"), u


def test_polynomial_unstable_at_vanishing_viscosity(ks):
    # the stable speed collapses as nu -> 0
    s_small = st.max_stable_speed(1e-6, 0.0, ks, kind="poly2", iters=20)
    s_mid = st.max_stable_speed(1e-3, 0.0, ks, kind="poly2", iters=20)
    assert s_small < s_mid < 1.0 - CS + 1e-4
