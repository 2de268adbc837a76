"""Pins of the oracle's effective-viscosity factor A and relaxation frequency.

* A of the entropic equilibrium (eq. entropic_bulk) is checked against the
  paper's general expression eq. (entorpic_bulk), with P*_xx and its
  derivatives taken by finite differences of the oracle's own equilibrium
  (P* = sum (c - u)^2 f^eq - rho varsigma^2); the compressibility error of
  eq. (entorpic_bulk_2) must vanish (eq. bulk_compressibility_error_entropic).
* Limits stated in Sec. "1-D lattice: Bulk viscosity": A -> 0 as u -> 1,
  A positive, second-order approach to 1 as u -> 0; polynomial A
  (eq. LBGK_bulk) loses positivity beyond |u| = varsigma sqrt(2/3)
  (eq. bulk_poly_positivity).
* beta (eq. relaxation_frequency) gives 2 beta = 1/tau for nu = varsigma^2
  (tau - 1/2); the corrected beta (eq. redefined_relaxation rate) stays in
  (0, 1] for the entropic equilibrium and leaves it for polynomial A
  (Sec. "Rescaling bulk viscosity").
"""
import numpy as np
import pytest

import oracle

CS2 = 1.0 / 3.0


def _pstar(rho, u, kind="entropic"):
    f, _ = oracle.equilibrium(rho, np.array([u]), kind=kind)
    c, _ = oracle.lattice(1)
    return np.sum((c[:, 0] - u) ** 2 * f) - rho * CS2


def _general_A_B(rho, u, kind="entropic", h=1e-5):
    P = lambda r, v: _pstar(r, v, kind)
    dPu = (P(rho, u + h) - P(rho, u - h)) / (2 * h)
    dPr = (P(rho + h, u) - P(rho - h, u)) / (2 * h)
    A = (1 - 1.5 * u * u / CS2 - 1.5 / (rho * CS2) * u * dPu - dPu ** 2 / (2 * rho ** 2 * CS2)
         - dPr / (2 * CS2))
    B = -3 * u * dPr - CS2 / rho * dPu - dPu * dPr / rho - u ** 3
    return A, B


@pytest.mark.parametrize("rho", [0.6, 1.0, 1.9])
def test_entropic_A_matches_general_expression_and_B_vanishes(rho):
    for u in np.linspace(-0.95, 0.95, 39):
        A_gen, B_gen = _general_A_B(rho, u)
        assert abs(oracle.bulk_A(u) - A_gen) < 2e-8, u
        assert abs(B_gen) < 2e-8, u


@pytest.mark.parametrize("kind", ["poly2", "product"])
def test_polynomial_A_matches_general_expression(kind):
    """With P* = 0 the general expression reduces to eq. (LBGK_bulk) and B = -u^3."""
    for u in np.linspace(-0.4, 0.4, 17):
        A_gen, B_gen = _general_A_B(1.0, u, kind=kind)
        assert abs(oracle.bulk_A(u, kind="poly2") - A_gen) < 2e-8
        assert abs(B_gen + u ** 3) < 2e-8


def test_entropic_A_limits_and_shape():
    us = np.linspace(0.0, 0.9999, 2001)
    A = np.array([oracle.bulk_A(u) for u in us])
    assert A[0] == 1.0
    assert np.all(A > 0) and np.all(A <= 1)
    assert np.all(np.diff(A) < 0)  # monotone decreasing in |u|
    assert oracle.bulk_A(0.9999) < 1e-3
    for u in us[1:50]:
        assert oracle.bulk_A(-u) == oracle.bulk_A(u)
    # second-order approach to the nominal viscosity: (1 - A)/u^2 -> 9/2
    small = np.array([1e-2, 5e-3, 2.5e-3])
    ratio = np.array([(1 - oracle.bulk_A(u)) / u ** 2 for u in small])
    assert np.allclose(ratio, 4.5, rtol=1e-3)


def test_polynomial_A_positivity_bound():
    bound = np.sqrt(CS2 * 2.0 / 3.0)
    assert oracle.bulk_A(bound * 0.999, kind="poly2") > 0
    assert oracle.bulk_A(bound * 1.001, kind="poly2") < 0


@pytest.mark.parametrize("tau", [0.5001, 0.51, 0.8, 1.0, 1.7])
def test_beta_uncorrected(tau):
    for D in (1, 2, 3):
        assert 2 * oracle.beta(tau, np.full(D, 0.3)) == pytest.approx(1.0 / tau, rel=1e-15)


def test_beta_corrected():
    tau = 0.51
    nu = CS2 * (tau - 0.5)
    # rest state: correction is the identity (A(0) = 1)
    assert oracle.beta(tau, np.zeros(2), corr="min") == oracle.beta(tau, np.zeros(2))
    # 1-D: beta = 1 / (2 nu / (A varsigma^2) + 1)
    for u in (0.05, -0.3, 0.9):
        A = oracle.bulk_A(u)
        assert oracle.beta(tau, np.array([u]), corr="min") == pytest.approx(1 / (2 * nu / (A * CS2) + 1), rel=1e-15)
    # multi-D min reading: the axis with the largest |u| sets A
    u = np.array([0.1, -0.2])
    assert oracle.beta(tau, u, corr="min") == oracle.beta(tau, np.array([-0.2]), corr="min")
    # entropic corrected beta stays in (0, 1] on |u| < 1
    for tau in (0.5001, 0.6, 1.0, 3.0):
        for ux in np.linspace(-0.999, 0.999, 101):
            b = oracle.beta(tau, np.array([ux, 0.5 * ux]), corr="min")
            assert 0 < b <= 1
    # polynomial correction leaves [0, 1] once A < 0
    b = oracle.beta(0.6, np.array([0.6]), corr="min", kind="poly2")
    assert not (0 <= b <= 1)


def test_beta_corrected_product_rule():
    """The oracle's second reading of a multi-D node's A (corr "product"):
    A = prod_alpha A(u_alpha), each factor the 1-D A of eq. (entorpic_bulk)."""
    tau = 0.51
    nu = CS2 * (tau - 0.5)
    # one non-zero component: both readings reduce to the 1-D A (A(0) = 1 exactly)
    for u in ([0.3, 0.0], [0.0, -0.7], [0.0, 0.0, 0.45], [0.9]):
        u = np.array(u)
        assert oracle.beta(tau, u, corr="product") == oracle.beta(tau, u, corr="min")
    # two components: the product of the general expression's A at each (finite
    # differences of P*), not the smaller one
    A1, _ = _general_A_B(1.0, 0.1)
    A2, _ = _general_A_B(1.0, -0.2)
    expected = 1.0 / (2.0 * nu / (A1 * A2 * CS2) + 1.0)
    assert oracle.beta(tau, np.array([0.1, -0.2]), corr="product") == pytest.approx(expected, rel=1e-7)
    A3, _ = _general_A_B(1.0, 0.35)
    expected3 = 1.0 / (2.0 * nu / (A1 * A2 * A3 * CS2) + 1.0)
    assert oracle.beta(tau, np.array([0.1, -0.2, 0.35]), corr="product") == pytest.approx(expected3, rel=1e-7)
    # A(u) <= 1, so the product never exceeds the min: the product rule relaxes
    # more slowly; symmetric under axis permutations and sign changes
    rng = np.random.default_rng(5)
    for _ in range(200):
        u = rng.uniform(-0.95, 0.95, 3)
        b_prod = oracle.beta(tau, u, corr="product")
        assert 0 < b_prod <= oracle.beta(tau, u, corr="min")
        assert oracle.beta(tau, u[::-1] * np.array([1, -1, 1]), corr="product") == pytest.approx(b_prod, rel=1e-15)
