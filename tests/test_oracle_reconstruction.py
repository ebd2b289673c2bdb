"""Pins of the oracle's reconstruction (Sec. 2.1/2.2 Steps 1-3, Appendix A)
against the defining conditions, polynomial exactness and closed forms."""
import numpy as np
import pytest

import oracle as O
import bruteforce as BF

RNG = np.random.default_rng(12345)


def p1d(weights=O.W_BETA, gam=None):
    return O.Problem(dim=1, flux=O.ADVECTION, nx=8, weights=weights,
                     gamma_lin=gam or (0.995, 0.0025, 0.0025))


def p2d(weights=O.W_BETA, gam=None, Q=2):
    return O.Problem(dim=2, flux=O.ADVECTION, nx=8, ny=8, weights=weights, gauss_q=Q,
                     gamma_lin=gam or (0.99, 0.0025, 0.0025, 0.0025, 0.0025))


# ---------------------------------------------------------------- 1D ------

def test_1d_coefficients_solve_defining_conditions():
    """Appendix A (1D) equals the unique solution of the Step 1 conditions."""
    p = p1d()
    for _ in range(20):
        ub = RNG.normal(size=3)
        vb = RNG.normal(size=2)
        dx = RNG.uniform(0.01, 2.0)
        r = O.recon_1d(p, ub, vb, dx)
        ref = BF.p0_1d(ub, dx * vb[0], dx * vb[1])
        np.testing.assert_allclose(r["c0"], ref, rtol=0, atol=1e-13 * (1 + np.abs(ref).max()))
        assert r["c1"][0] == ub[1] and r["c1"][1] == ub[1] - ub[0]
        assert r["c2"][0] == ub[1] and r["c2"][1] == ub[2] - ub[1]


@pytest.mark.parametrize("deg", range(5))
def test_1d_p0_exact_for_quartics(deg):
    """Data of a polynomial of degree <= 4 is reproduced exactly by p0, and by
    the whole reconstruction in linear-weight mode (point values, u_x, v-hat)."""
    coef = RNG.normal(size=deg + 1)
    P = np.polynomial.Polynomial(coef)
    Pi, dP = P.integ(), P.deriv()
    ub = [Pi(k + 0.5) - Pi(k - 0.5) for k in (-1, 0, 1)]
    dx = 0.37
    vb = [(P(k + 0.5) - P(k - 0.5)) / dx for k in (-1, 1)]
    r = O.recon_1d(p1d(O.W_LINEAR), ub, vb, dx)
    full = np.zeros(5)
    full[:deg + 1] = coef
    np.testing.assert_allclose(r["c0"], full, atol=1e-13)
    assert abs(r["u_right"] - P(0.5)) < 1e-13 and abs(r["u_left"] - P(-0.5)) < 1e-13
    assert abs(r["ux_right"] - dP(0.5) / dx) < 1e-12
    assert abs(r["ux_left"] - dP(-0.5) / dx) < 1e-12
    assert abs(r["vhat"] - (P(0.5) - P(-0.5)) / dx) < 1e-12


def test_1d_linear_data_gives_linear_weights():
    """u = xi: every smoothness indicator equals 1, tau = 0, omega = gamma and
    the reconstruction is exact (u(+-1/2) = +-1/2, v-hat = 1)."""
    ub = [-1.0, 0.0, 1.0]
    for w in (O.W_PAPER, O.W_BETA, O.W_BETA2):
        r = O.recon_1d(p1d(w), ub, [1.0, 1.0], 1.0)
        np.testing.assert_allclose(r["beta"], [1, 1, 1], atol=1e-15)
        np.testing.assert_allclose(r["omega"], [0.995, 0.0025, 0.0025], atol=1e-15)
        assert abs(r["u_right"] - 0.5) < 1e-15 and abs(r["u_left"] + 0.5) < 1e-15
        assert abs(r["vhat"] - 1.0) < 1e-14


def test_1d_quadratic_worked_example():
    """u = xi^2 (dx = 1): p0 = xi^2 exactly, so beta0 = (2! * 1)^2 = 4 and the
    one-sided slopes give beta1 = beta2 = 1; tau = 3.  The weights then follow
    the closed form gamma_m (1 + 9 / (beta_m + eps)) / sum, and by symmetry
    v-hat = 0 and u(+1/2) = u(-1/2)."""
    ub = [13 / 12, 1 / 12, 13 / 12]     # averages of xi^2 over the three cells
    vb = [-2.0, 2.0]
    g = np.array([0.995, 0.0025, 0.0025])
    eps = 1e-8
    for mode, den in ((O.W_BETA, np.array([4.0, 1.0, 1.0]) + eps),
                      (O.W_BETA2, np.array([16.0, 1.0, 1.0]) + eps)):
        r = O.recon_1d(p1d(mode), ub, vb, 1.0)
        np.testing.assert_allclose(r["c0"], [0, 0, 1, 0, 0], atol=1e-15)
        np.testing.assert_allclose(r["beta"], [4, 1, 1], atol=1e-14)
        wt = g * (1 + 9.0 / den)
        np.testing.assert_allclose(r["omega"], wt / wt.sum(), rtol=1e-14)
        w = wt / wt.sum()
        # u_i = w0/g0 * xi^2 + (constant part): value at +-1/2
        const = w[0] * (0 - g[1] / g[0] * ub[1] - g[2] / g[0] * ub[1]) + (w[1] + w[2]) * ub[1]
        expect = w[0] / g[0] * 0.25 + const
        assert abs(r["u_right"] - expect) < 1e-14 and abs(r["u_left"] - expect) < 1e-14
        assert abs(r["vhat"]) < 1e-14
    # the closed form above for the beta + eps form, as a fixed number
    r = O.recon_1d(p1d(O.W_BETA), ub, vb, 1.0)
    assert abs(r["u_right"] - 0.248287019432038) < 1e-12


def test_1d_step_discontinuity_drops_the_quartic():
    """A jump between cells i and i+1: the weights move onto the smooth left
    linear stencil (omega_1 -> 1), as the essentially non-oscillatory design
    requires."""
    r = O.recon_1d(p1d(O.W_BETA), [0.0, 0.0, 1.0], [0.0, 0.0], 1.0)
    assert r["omega"][1] > 0.9999999 and r["omega"][0] < 1e-7 and r["omega"][2] < 1e-7
    assert abs(r["u_right"]) < 1e-6 and abs(r["u_left"]) < 1e-6


# ---------------------------------------------------------------- 2D ------

def _q_from(ub9, v4, w4):
    return np.concatenate([ub9, v4, w4])


def test_2d_coefficients_are_face_neighbour_constrained_least_squares():
    """Appendix A (2D) equals the equality-constrained least-squares solution
    that fits the derivative averages of the four face neighbours."""
    p = p2d()
    for _ in range(20):
        ub9 = RNG.normal(size=9)
        v4 = RNG.normal(size=4)
        w4 = RNG.normal(size=4)
        r = O.recon_2d(p, _q_from(ub9, v4, w4))
        ref = BF.p0_2d(ub9, v4, w4)
        np.testing.assert_allclose(r["c0"], ref, atol=1e-12 * (1 + np.abs(ref).max()))


def test_2d_coefficients_differ_from_eight_neighbour_least_squares():
    """The text of Step 1 mentions all neighbours; the printed coefficients do
    not match that fit (they match the face-neighbour fit above)."""
    ub9 = RNG.normal(size=9)
    v8 = RNG.normal(size=8)
    w8 = RNG.normal(size=8)
    # face neighbours W, E, S, N sit at positions 3, 4, 1, 6 of the 8
    v4 = v8[[3, 4, 1, 6]]
    w4 = w8[[3, 4, 1, 6]]
    r = O.recon_2d(p2d(), _q_from(ub9, v4, w4))
    ref8 = BF.p0_2d(ub9, v8, w8, neighbours="all8")
    assert np.abs(r["c0"] - ref8).max() > 1e-3


@pytest.mark.parametrize("l", range(15))
def test_2d_p0_exact_on_every_monomial(l):
    """Each monomial of degree <= 4 is reproduced exactly by p0, and in linear
    mode the reconstruction's edge values, derivatives and hats are exact."""
    m, n = BF.MN[l]
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    ub9 = [BF.integ(m, a - .5, a + .5) * BF.integ(n, b - .5, b + .5) for a, b in cells]
    nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    v4 = [((a + .5) ** m - (a - .5) ** m) * BF.integ(n, b - .5, b + .5) if m else 0.0
          for a, b in nb]
    w4 = [((b + .5) ** n - (b - .5) ** n) * BF.integ(m, a - .5, a + .5) if n else 0.0
          for a, b in nb]
    r = O.recon_2d(p2d(O.W_LINEAR), _q_from(ub9, v4, w4))
    expect = np.zeros(15)
    expect[l] = 1.0
    np.testing.assert_allclose(r["c0"], expect, atol=1e-13)
    np.testing.assert_allclose(r["C"], expect, atol=1e-13)
    vh = m * BF.integ(m - 1, -.5, .5) * BF.integ(n, -.5, .5) if m else 0.0
    wh = n * BF.integ(m, -.5, .5) * BF.integ(n - 1, -.5, .5) if n else 0.0
    assert abs(r["vhat"] - vh) < 1e-13 and abs(r["what"] - wh) < 1e-13
    for x, y in ((0.5, 0.3), (-0.5, -0.2), (0.1, 0.5), (-0.4, -0.5)):
        val = O.poly2d_eval(r["C"], x, y)
        ref = BF.eval2(expect, x, y)
        np.testing.assert_allclose(val, ref, atol=1e-13)


def test_2d_basis_order_is_xi_first():
    """Read with the other order of each degree (eta^n first) the printed
    coefficients are no longer exact: the xi-first order is the right one."""
    # data of eta^2 read back as coefficients: position 5 (eta^2), not 3 (xi^2)
    m, n = 0, 2
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    ub9 = [BF.integ(m, a - .5, a + .5) * BF.integ(n, b - .5, b + .5) for a, b in cells]
    nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    w4 = [((b + .5) ** n - (b - .5) ** n) * BF.integ(m, a - .5, a + .5) for a, b in nb]
    r = O.recon_2d(p2d(), _q_from(ub9, [0.0] * 4, w4))
    assert abs(r["c0"][5] - 1.0) < 1e-13 and abs(r["c0"][3]) < 1e-13


def test_2d_linear_data_gives_linear_weights():
    """u = xi + 2 eta: tau = 0, omega = gamma, v-hat = 1, w-hat = 2."""
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    ub9 = [a + 2.0 * b for a, b in cells]
    q = _q_from(ub9, [1.0] * 4, [2.0] * 4)
    for mode in (O.W_PAPER, O.W_BETA, O.W_BETA2):
        r = O.recon_2d(p2d(mode), q)
        np.testing.assert_allclose(r["beta"], [5.0] * 5, atol=1e-13)
        np.testing.assert_allclose(r["omega"], [0.99] + [0.0025] * 4, atol=1e-15)
        assert abs(r["vhat"] - 1.0) < 1e-14 and abs(r["what"] - 2.0) < 1e-14


def test_2d_quadratic_worked_example():
    """u = xi^2: beta0 = 4, every linear stencil has slope +-1 in xi and 0 in
    eta so beta_m = 1, tau = 3; weights in closed form; v-hat = w-hat = 0."""
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    ub9 = [BF.integ(2, a - .5, a + .5) for a, b in cells]
    v4 = [((a + .5) ** 2 - (a - .5) ** 2) for a, b in [(-1, 0), (1, 0), (0, -1), (0, 1)]]
    q = _q_from(ub9, v4, [0.0] * 4)
    g = np.array([0.99, 0.0025, 0.0025, 0.0025, 0.0025])
    for mode, den in ((O.W_BETA, np.array([4.0, 1, 1, 1, 1]) + 1e-8),
                      (O.W_BETA2, np.array([16.0, 1, 1, 1, 1]) + 1e-8)):
        r = O.recon_2d(p2d(mode), q)
        np.testing.assert_allclose(r["beta"], [4, 1, 1, 1, 1], atol=1e-13)
        wt = g * (1 + 9.0 / den)
        np.testing.assert_allclose(r["omega"], wt / wt.sum(), rtol=1e-13)
        assert abs(r["vhat"]) < 1e-14 and abs(r["what"]) < 1e-14
    r = O.recon_2d(p2d(O.W_BETA2), q)
    # the closed form for the beta^2 + eps form as fixed numbers: omega_0, and
    # u, u_xi at the Gauss point (1/2, 1/(2 sqrt 3)) of the right face
    assert abs(r["omega"][0] - 0.939278937882) < 1e-11
    val = O.poly2d_eval(r["C"], 0.5, 0.5 / np.sqrt(3.0))
    assert abs(val[0] - 0.241461100654) < 1e-11
    assert abs(val[1] - 0.948766603921) < 1e-11


def test_2d_mixed_term_invisible_to_linear_stencils():
    """u = xi*eta: beta0 = 1 but all linear slopes vanish (beta_m = 0), so
    tau = 1 and the weight of p0 collapses -- an expected property."""
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    ub9 = [a * b for a, b in cells]
    nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    q = _q_from(ub9, [b for a, b in nb], [a for a, b in nb])
    r = O.recon_2d(p2d(O.W_BETA2), q)
    np.testing.assert_allclose(r["beta"], [1, 0, 0, 0, 0], atol=1e-14)
    assert r["omega"][0] < 3e-6
