"""Pin of the oracle's one departure from plain FP64: the entropic equilibrium
evaluated in extended precision and rounded once per population.

Sec. "Discrete entropic equilibrium construction" builds f^eq so that its mass
and momentum equal rho and rho u exactly.  Evaluated in double, the multiplier
form w_i X^{-1} prod Z_alpha^{c_ia} misses the momentum constraint by a few
units in the last place, with a sign that repeats from step to step, so
repeated collisions act as a small spurious force.  Near tau = 1/2 nothing
damps it and the velocity drifts linearly in time.

Three runs of one of the batched workload's shear waves (D2Q9 periodic,
u_x = a sin(2 pi y / ny), a = 0.01, nu = 1e-5, 2000 steps; the field does not
depend on x, so one column stands for any width) are compared here, each
written in numpy independently of the C oracle:

  H   every quantity in x87 extended precision (state, moments, equilibrium,
      relaxation, streaming): the trajectory of the scheme itself, with
      rounding ~2^11 times smaller than double's;
  Dd  every quantity in double, the equilibrium in the multiplier form;
  X   double state, moments and relaxation, the equilibrium in extended
      precision rounded once per population: the scheme the oracle states.

The oracle must equal X bitwise; Dd must drift past the 1e-12 FP64 budget
linearly in time, while the oracle stays inside it and at least 10 times
closer to H than Dd.  What remains of the oracle's distance to H is the
rounding of the double state itself.
"""
import numpy as np
import pytest

import oracle

LD = np.longdouble


def _d2q9(dtype):
    c = np.array([(cx, cy) for cx in (-1, 0, 1) for cy in (-1, 0, 1)])
    one = dtype(1)
    w1 = {-1: one / 6, 0: one * 2 / 3, 1: one / 6}
    w = np.array([w1[cx] * w1[cy] for cx, cy in c], dtype=dtype)
    return c, w


def _multiplier_feq(c, w, rho, ux, uy, out_dtype):
    """eq. (Entropic_isothermal_EDF): f_i = w_i X^{-1} prod Z^{c_ia}, computed in
    the dtype of rho/u and cast to out_dtype."""
    one = rho.dtype.type(1)
    cs2 = one / 3
    xinv = rho.copy()
    Z = []
    for ua in (ux, uy):
        root = np.sqrt(ua * ua / cs2 + one)
        Z.append((2 * ua + root) / (one - ua))
        xinv = xinv * (2 - root)
    out = []
    for i, (cx, cy) in enumerate(c):
        p = np.ones_like(rho)
        for ca, Za in zip((cx, cy), Z):
            if ca == 1:
                p = p * Za
            elif ca == -1:
                p = p / Za
        out.append((rho.dtype.type(w[i]) * xinv * p).astype(out_dtype))
    return np.array(out)


def _moments(c, f):
    rho = np.zeros_like(f[0])
    jx = np.zeros_like(rho)
    jy = np.zeros_like(rho)
    for i in range(9):
        rho += f[i]
        jx += c[i, 0] * f[i]
        jy += c[i, 1] * f[i]
    return rho, jx / rho, jy / rho


def _run(rho0, u0, tau, steps, state, eq):
    """LBGK steps (Sec. "Basic concepts") with the state in `state` precision and
    the equilibrium evaluated in `eq` precision; push streaming, periodic."""
    c, w = _d2q9(state)
    _, w_eq = _d2q9(eq)
    if state is np.float64:
        w_eq = w.astype(eq)  # the oracle's weights are the double ones
    two_beta = state(1) / state(tau)

    def feq(rho, ux, uy):
        return _multiplier_feq(c, w_eq, rho.astype(eq), ux.astype(eq), uy.astype(eq), state)

    f = feq(rho0.astype(state), u0[0].astype(state), u0[1].astype(state))
    for _ in range(steps):
        rho, ux, uy = _moments(c, f)
        f = f + two_beta * (feq(rho, ux, uy) - f)
        for i in range(9):
            f[i] = np.roll(np.roll(f[i], c[i, 0], axis=1), c[i, 1], axis=0)
    rho, ux, uy = _moments(c, f)
    return rho, np.array([ux, uy])


def _rel(a, b):
    a = np.asarray(a, dtype=np.float64)
    b = np.asarray(b, dtype=np.float64)
    return float(np.max(np.abs(a - b)) / np.max(np.abs(b)))


def _shear_wave(ny=64, amp=0.01):
    y = np.arange(ny)
    rho0 = np.ones((ny, 1))
    u0 = np.zeros((2, ny, 1))
    u0[0] = amp * np.sin(2 * np.pi * y / ny)[:, None]
    return rho0, u0


def test_extended_equilibrium_keeps_the_oracle_on_the_trajectory():
    assert np.finfo(LD).nmant >= 63, "needs x87 extended precision for the high-precision run"
    rho0, u0 = _shear_wave()
    tau = 0.5 + 3 * 1e-5
    errs = {}
    for steps in (500, 2000):
        _, u_h = _run(rho0, u0, tau, steps, LD, LD)
        _, u_dd = _run(rho0, u0, tau, steps, np.float64, np.float64)
        r_x, u_x = _run(rho0, u0, tau, steps, np.float64, LD)
        r_o, u_o, bad = oracle.run(rho0, u0, tau, steps)
        assert bad == 0
        # the oracle computes exactly the stated scheme
        assert np.array_equal(r_o, r_x) and np.array_equal(u_o, u_x)
        errs[steps] = (_rel(u_dd, u_h), _rel(u_o, u_h))
    dd, o = errs[2000]
    assert dd > 5e-12, errs          # the double multiplier form leaves the 1e-12 budget
    assert errs[2000][0] > 3.5 * errs[500][0], errs  # linearly in time
    assert o < 1e-12, errs           # the oracle stays inside it
    assert dd > 10 * o, errs


def test_oracle_meets_the_momentum_constraint_to_population_rounding():
    """Single nodes: the momentum error sum_i c_ix f_i - rho u_x, taken exactly
    on the rounded populations, in units of rho * 2^-52.  Rounding each f_i to
    nearest moves it by at most half an ulp, at most 2^-53 f_i, and the f_i with
    c_x != 0 sum to less than rho, so an equilibrium that is exact before its
    one rounding misses the constraint by at most 1/2 unit.  The oracle stays
    inside that bound; the double multiplier form does not."""
    rng = np.random.default_rng(7)
    c, w = _d2q9(np.float64)
    n = 4000
    rho = rng.uniform(0.9, 1.1, n)
    ux = rng.uniform(-0.2, 0.2, n)
    uy = rng.uniform(-0.2, 0.2, n)
    f_dd = _multiplier_feq(c, w, rho, ux, uy, np.float64)
    f_o = np.array([oracle.equilibrium(r, np.array([a, b]))[0] for r, a, b in zip(rho, ux, uy)]).T
    # exact target rho u_x, and the momentum of the rounded populations, in extended precision
    target = rho.astype(LD) * ux.astype(LD)

    def err(f):
        j = np.zeros(n, dtype=LD)
        for i in range(9):
            j += c[i, 0] * f[i].astype(LD)
        return ((j - target) / (rho.astype(LD) * LD(np.finfo(np.float64).eps))).astype(np.float64)

    e_dd, e_o = err(f_dd), err(f_o)
    assert np.max(np.abs(e_o)) <= 0.5 + 1e-3
    assert np.max(np.abs(e_dd)) > 0.6
    assert np.std(e_dd) > 2 * np.std(e_o)


@pytest.mark.parametrize("steps", [1, 7])
def test_high_precision_runner_matches_the_oracle_on_short_runs(steps):
    """The numpy runners here agree with the oracle where rounding has no time
    to accumulate (guards the test's own scheme against a slip)."""
    rho0, u0 = _shear_wave(ny=16, amp=0.1)
    u0[1] = 0.03 * np.cos(2 * np.pi * np.arange(16) / 16)[:, None]
    _, u_h = _run(rho0, u0, 0.6, steps, LD, LD)
    _, u_o, _ = oracle.run(rho0, u0, 0.6, steps)
    assert _rel(u_o, u_h) < 1e-14
