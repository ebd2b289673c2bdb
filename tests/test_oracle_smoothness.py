"""Pins of the oracle's classical smoothness indicator, the option that
replaces the paper's moment-based indicator of p0 by the integral form the
paper prints for comparison (eq. smoothness-indicator-typical and its 2D
form).  In cell units it is the sum over derivative orders of the integrals
of the squared derivatives over the cell."""
import numpy as np
import numpy.polynomial.polynomial as npp
import pytest

import oracle as O
from paper_2607_24325_amd import workloads as W

RNG = np.random.default_rng(11)
MEXP = [0, 1, 0, 2, 1, 0, 3, 2, 1, 0, 4, 3, 2, 1, 0]
NEXP = [0, 0, 1, 0, 1, 2, 0, 1, 2, 3, 0, 1, 2, 3, 4]


def test_1d_monomials_by_hand():
    # xi: 1;  xi^2: (2 xi)^2 -> 1/3, 2^2 -> 4;  xi^3: 9/80 + 3 + 36;
    # xi^4: 1/28 + 9/5 + 48 + 576;  xi + xi^3: (1 + 3 xi^2)^2 -> 1 + 1/2 + 9/80, + 3 + 36
    cases = [([0, 1, 0, 0, 0], 1.0), ([0, 0, 1, 0, 0], 13.0 / 3.0),
             ([0, 0, 0, 1, 0], 9.0 / 80.0 + 39.0), ([0, 0, 0, 0, 1], 1 / 28 + 9 / 5 + 624),
             ([0, 1, 0, 1, 0], 1.5 + 9.0 / 80.0 + 39.0), ([7.0, 0, 0, 0, 0], 0.0)]
    for c, want in cases:
        assert O.smoothness_classical(c) == pytest.approx(want, rel=1e-14, abs=1e-15)


def test_2d_monomials_by_hand():
    def c2(**kw):
        c = np.zeros(15)
        for k, v in kw.items():
            c[int(k[1:])] = v
        return c
    # xi eta: eta^2 and xi^2 integrate to 1/12 each, the mixed derivative to 1
    assert O.smoothness_classical(c2(k4=1.0)) == pytest.approx(1 / 6 + 1, rel=1e-14)
    # xi^2 eta^2: 2 (4/960) + 2 (4/80) + 16/144 + 2 (16/12) + 16
    want = 2 * 4 / 960 + 2 * 4 / 80 + 16 / 144 + 2 * 16 / 12 + 16
    assert O.smoothness_classical(c2(k12=1.0)) == pytest.approx(want, rel=1e-14)


def _classical_exact_numpy(c):
    """independent route: numpy 2D polynomial derivatives and exact
    antiderivatives over [-1/2, 1/2]^2"""
    P = np.zeros((5, 5))
    for k in range(15):
        P[MEXP[k], NEXP[k]] = c[k]
    total = 0.0
    for m in range(5):
        for n in range(5 - m):
            if m + n == 0:
                continue
            D = npp.polyder(npp.polyder(P, m, axis=0), n, axis=1)
            Dp = np.zeros((D.shape[0] * 2, D.shape[1] * 2))   # D squared
            for a in range(D.shape[0]):
                for b in range(D.shape[1]):
                    Dp[a:a + D.shape[0], b:b + D.shape[1]] += D[a, b] * D
            I = npp.polyint(npp.polyint(Dp, 1, lbnd=-0.5, axis=0), 1, lbnd=-0.5, axis=1)
            total += npp.polyval2d(0.5, 0.5, I)
    return total


def test_2d_matches_exact_integration_on_random_quartics():
    for _ in range(20):
        c = RNG.normal(size=15)
        assert O.smoothness_classical(c) == pytest.approx(_classical_exact_numpy(c), rel=1e-12)


def test_structure():
    """a 2D polynomial of xi alone has the 1D value; x <-> y symmetry;
    quadratic scaling; constants do not count; linear polynomials give the
    moment value (squared slopes)"""
    for _ in range(10):
        c1 = RNG.normal(size=5)
        c2 = np.zeros(15)
        for k in range(15):
            if NEXP[k] == 0:
                c2[k] = c1[MEXP[k]]
        assert O.smoothness_classical(c2) == pytest.approx(O.smoothness_classical(c1), rel=1e-13)
        c = RNG.normal(size=15)
        ct = np.zeros(15)
        for k in range(15):
            j = [i for i in range(15) if MEXP[i] == NEXP[k] and NEXP[i] == MEXP[k]][0]
            ct[j] = c[k]
        assert O.smoothness_classical(ct) == pytest.approx(O.smoothness_classical(c), rel=1e-13)
        assert O.smoothness_classical(3 * c) == pytest.approx(9 * O.smoothness_classical(c), rel=1e-13)
        c0 = c.copy()
        c0[0] += 5.0
        assert O.smoothness_classical(c0) == pytest.approx(O.smoothness_classical(c), rel=1e-13)
        lin = np.zeros(15)
        lin[1:3] = c[1:3]
        assert O.smoothness_classical(lin) == pytest.approx(c[1] ** 2 + c[2] ** 2, rel=1e-13)


def test_reconstruction_uses_the_selected_indicator():
    p = O.Problem(dim=1, flux=O.BURGERS, nx=8, weights=O.W_BETA, smoothness=O.BETA_CLASSICAL)
    r = O.recon_1d(p, [0.1, 0.5, 2.0], [0.3, -1.0], 0.1)
    assert r["beta"][0] == pytest.approx(O.smoothness_classical(r["c0"]), rel=1e-15)
    pm = O.Problem(dim=1, flux=O.BURGERS, nx=8, weights=O.W_BETA)
    rm = O.recon_1d(pm, [0.1, 0.5, 2.0], [0.3, -1.0], 0.1)
    assert np.allclose(rm["beta"][1:], r["beta"][1:]) and rm["beta"][0] != r["beta"][0]
    q = RNG.normal(size=17)
    p2 = O.Problem(dim=2, flux=O.BURGERS, nx=8, ny=8, weights=O.W_BETA,
                   smoothness=O.BETA_CLASSICAL)
    r2 = O.recon_2d(p2, q)
    assert r2["beta"][0] == pytest.approx(O.smoothness_classical(r2["c0"]), rel=1e-15)


def _advection_l1(n, smooth):
    spec, st = W.advection_1d(n)
    p = O.Problem(dim=1, flux=O.ADVECTION, nx=n, xlo=spec.xlo, xhi=spec.xhi, adv=spec.adv,
                  weights=O.W_BETA, smoothness=smooth)
    out, _ = O.run(p, st, 0.0, 2.0, 0.6, 5.0 / 3.0)
    return np.abs(out[0, 0, 0] - st[0, 0, 0]).mean()


def test_fifth_order_with_the_classical_indicator():
    """smooth advection to t = 2 (dt ~ dx^(5/3)): the classical indicator keeps
    fifth order, and its errors stay within a factor 2 of the moment form's"""
    e = [_advection_l1(n, O.BETA_CLASSICAL) for n in (40, 80, 160)]
    orders = np.log2(np.array(e[:-1]) / np.array(e[1:]))
    assert orders[-1] > 4.6, orders
    em = _advection_l1(160, O.BETA_MOMENT)
    assert 0.5 < e[-1] / em < 2.0, (e[-1], em)
