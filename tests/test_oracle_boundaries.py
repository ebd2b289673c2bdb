"""Pins of the oracle's boundary treatment, Euler flux derivatives and
Lax-Friedrichs speeds against an independent brute-force statement
(``bruteforce_sys``: numpy padding for the ghost cells, complex-step
Jacobians, spectral radii from ``np.linalg.eigvals``, Step 1 solved as
linear systems).

* Lax-Friedrichs speed (Sec. 2.1: alpha = max |f'(u)|; Sec. 2.2: separate
  alpha_x, alpha_y): the oracle's speed equals the spectral radius of the
  flux Jacobian, and states with a known sound speed give hand-checked
  values.
* Transmissive boundaries (the boundary type of the shock-tube examples of
  Sec. 3.2): every unknown of a ghost cell, the derivative averages
  included, is that of the nearest interior cell; 2D corners follow both
  axis maps.
* Per-stage speeds (an option of this library, not in the paper): each stage
  takes the spectral radius over its own input state.
"""
import numpy as np
import pytest

import oracle as O
import bruteforce_sys as B

RNG = np.random.default_rng(20261203)


def _euler_state_1d(n, rng):
    x = (np.arange(n) + 0.5) / n
    rho = 1.0 + 0.3 * np.sin(2 * np.pi * x) + 0.1 * rng.uniform(-1, 1, n)
    u = 0.4 * np.cos(2 * np.pi * x) + 0.2 * rng.uniform(-1, 1, n)
    p = 1.0 + 0.2 * rng.uniform(-1, 1, n)
    st = np.zeros((2, 3, 1, n))
    st[0, 0, 0] = rho
    st[0, 1, 0] = rho * u
    st[0, 2, 0] = p / 0.4 + 0.5 * rho * u * u
    st[1] = 0.5 * rng.uniform(-1, 1, (3, 1, n))
    return st


def _euler_state_2d(n, rng):
    rho = 1.0 + 0.3 * rng.uniform(-1, 1, (n, n))
    u = 0.5 * rng.uniform(-1, 1, (n, n))
    v = 0.5 * rng.uniform(-1, 1, (n, n))
    p = 1.0 + 0.3 * rng.uniform(-1, 1, (n, n))
    st = np.zeros((3, 4, n, n))
    st[0] = [rho, rho * u, rho * v, p / 0.4 + 0.5 * rho * (u * u + v * v)]
    st[1:] = 0.5 * rng.uniform(-1, 1, (2, 4, n, n))
    return st


def _scale_err(got, want):
    """largest error per (variable, component) plane relative to that plane's
    largest value"""
    ax = tuple(range(2, want.ndim))
    scale = np.abs(want).max(axis=ax, keepdims=True) + 1e-300
    return float((np.abs(got - want) / scale).max())


# ----------------------------------------------------------------- speeds

def test_speed_of_states_with_a_known_sound_speed():
    # gamma p / rho = 1 (rho = 1.4, p = 1) and = 4 (rho = 0.35, p = 1): c = 1, 2
    st = np.zeros((3, 4, 4, 4))
    st[0, 0] = 1.4
    st[0, 3] = 1.0 / 0.4           # p = 1 at rest
    # one cell moving with (0.5, -2) at c = 1, one at rest with c = 2
    st[0, 1, 1, 2] = 1.4 * 0.5
    st[0, 2, 1, 2] = 1.4 * -2.0
    st[0, 3, 1, 2] = 1.0 / 0.4 + 0.5 * 1.4 * (0.25 + 4.0)
    st[0, 0, 3, 0] = 0.35
    p = O.Problem(dim=2, flux=O.EULER, nx=4, ny=4)
    ax, ay = O.alpha(p, st)
    assert ax == pytest.approx(2.0, rel=1e-15)           # |0| + 2 beats |0.5| + 1
    assert ay == pytest.approx(3.0, rel=1e-15)           # |-2| + 1
    # 1D: moving right at 1.5 with c = 1
    st1 = np.zeros((2, 3, 1, 4))
    st1[0, 0] = 1.4
    st1[0, 1] = 1.4 * -1.5
    st1[0, 2] = 1.0 / 0.4 + 0.5 * 1.4 * 2.25
    p1 = O.Problem(dim=1, flux=O.EULER, nx=4)
    assert O.alpha(p1, st1)[0] == pytest.approx(2.5, rel=1e-15)


def test_speed_of_the_smooth_euler_example():
    # Sec. 3.1 Example 2: rho = 1 + 0.2 sin(pi x), velocity 1, p = 1; the
    # largest |u| + c is at the density minimum 0.8: 1 + sqrt(1.4 / 0.8)
    n = 64
    x = (np.arange(n) + 0.5) / n * 2.0
    rho = 1.0 + 0.2 * np.sin(np.pi * x)
    rho[n * 3 // 4 - 1] = 0.8      # a cell at the exact minimum
    st = np.zeros((2, 3, 1, n))
    st[0, 0, 0] = rho
    st[0, 1, 0] = rho
    st[0, 2, 0] = 1.0 / 0.4 + 0.5 * rho
    p = O.Problem(dim=1, flux=O.EULER, nx=n, xlo=0.0, xhi=2.0)
    assert O.alpha(p, st)[0] == pytest.approx(1.0 + np.sqrt(1.75), rel=1e-15)


@pytest.mark.parametrize("dim", [1, 2])
def test_speed_is_the_spectral_radius_of_the_flux_jacobian(dim):
    rng = np.random.default_rng(5 + dim)
    n = 6
    st = _euler_state_1d(n, rng) if dim == 1 else _euler_state_2d(n, rng)
    p = O.Problem(dim=dim, flux=O.EULER, nx=n, ny=1 if dim == 1 else n)
    ax, ay = O.alpha(p, st)
    bx, by = B.speeds(B.euler_flux, st)
    assert ax == pytest.approx(bx, rel=1e-13)
    if dim == 2:
        assert ay == pytest.approx(by, rel=1e-13)
        assert ax != pytest.approx(ay, rel=1e-6)   # the two directions differ


@pytest.mark.parametrize("bad", ["rho_zero", "rho_negative", "p_negative", "nan"])
def test_speed_rejects_non_admissible_states(bad):
    rng = np.random.default_rng(3)
    st = _euler_state_2d(4, rng)
    if bad == "rho_zero":
        st[0, :, 2, 1] = [0.0, 0.0, 0.0, 1.0]
    elif bad == "rho_negative":
        st[0, 0, 2, 1] = -0.5
    elif bad == "p_negative":
        st[0, 3, 2, 1] = 0.5 * (st[0, 1, 2, 1] ** 2 + st[0, 2, 2, 1] ** 2) / st[0, 0, 2, 1] - 1e-3
    else:
        st[0, 2, 2, 1] = np.nan
    p = O.Problem(dim=2, flux=O.EULER, nx=4, ny=4)
    with pytest.raises(O.OracleError, match="cell 9"):    # j = 2, i = 1
        O.alpha(p, st)


def test_jacobian_vector_products_equal_the_complex_step():
    rng = np.random.default_rng(11)
    for dim in (1, 2):
        K = 3 if dim == 1 else 4
        p = O.Problem(dim=dim, flux=O.EULER, nx=4, ny=1 if dim == 1 else 4)
        for _ in range(5):
            st = _euler_state_2d(1, rng) if dim == 2 else _euler_state_1d(1, rng)
            U = st[0, :, 0, 0]
            V = rng.uniform(-1, 1, K)
            for d in range(dim):
                f, jv = O.flux(p, d, U, V)
                np.testing.assert_allclose(f, B.euler_flux(U, d), rtol=1e-14, atol=1e-14)
                np.testing.assert_allclose(jv, B.jvp(B.euler_flux, U, V, d), rtol=1e-13,
                                           atol=1e-13)


# ------------------------------------------------------ boundary treatment

def _oracle_1d(flux, n, bc, **kw):
    return O.Problem(dim=1, flux=flux, nx=n, xlo=0.0, xhi=1.0, bc_x=bc, weights=O.W_BETA,
                     **kw)


@pytest.mark.parametrize("bc", [O.PERIODIC, O.TRANSMISSIVE])
@pytest.mark.parametrize("flux", ["burgers", "euler"])
@pytest.mark.parametrize("n", [5, 7])
def test_1d_operator_matches_bruteforce(flux, bc, n):
    rng = np.random.default_rng(100 * n + bc)
    if flux == "euler":
        st = _euler_state_1d(n, rng)
        F, fl = B.euler_flux, O.EULER
    else:
        st = np.zeros((2, 1, 1, n))
        st[0, 0, 0] = 0.5 + rng.uniform(-1, 1, n)
        st[1, 0, 0] = rng.uniform(-2, 2, n)
        F, fl = B.scalar_flux("burgers"), O.BURGERS
    p = _oracle_1d(fl, n, bc)
    ax, _ = O.alpha(p, st)
    bx, _ = B.speeds(F, st)
    assert ax == pytest.approx(bx, rel=1e-13)
    L, Uh = O.rhs(p, st, ax)
    Lb, Uhb = B.rhs_1d(F, st, p.dx, ax, p.gamma_lin, p.eps, bc)
    assert _scale_err(L, Lb) < 1e-11
    assert _scale_err(Uh, Uhb) < 1e-11


@pytest.mark.parametrize("bcs", [(O.TRANSMISSIVE, O.TRANSMISSIVE), (O.TRANSMISSIVE, O.PERIODIC),
                                 (O.PERIODIC, O.TRANSMISSIVE)])
@pytest.mark.parametrize("flux", ["burgers", "euler"])
def test_2d_operator_matches_bruteforce(flux, bcs):
    n = 5
    rng = np.random.default_rng(7 + 3 * bcs[0] + bcs[1])
    if flux == "euler":
        st = _euler_state_2d(n, rng)
        F, fl = B.euler_flux, O.EULER
    else:
        st = np.zeros((3, 1, n, n))
        st[0, 0] = 0.5 + rng.uniform(-1, 1, (n, n))
        st[1:, 0] = rng.uniform(-2, 2, (2, n, n))
        F, fl = B.scalar_flux("burgers"), O.BURGERS
    p = O.Problem(dim=2, flux=fl, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.25,
                  bc_x=bcs[0], bc_y=bcs[1], gauss_q=2, weights=O.W_BETA)
    ax, ay = O.alpha(p, st)
    L, Uh = O.rhs(p, st, ax, ay)
    Lb, Uhb = B.rhs_2d(F, st, p.dx, p.dy, ax, ay, p.gamma_lin, p.eps, False, 2, *bcs)
    assert _scale_err(L, Lb) < 1e-11
    assert _scale_err(Uh, Uhb) < 1e-11


def test_transmissive_ghost_derivatives_matter():
    """The transmissive pin can see the ghost derivatives: zeroing them (a
    plausible misreading) moves the brute-force operator well beyond the bar
    that the oracle meets."""
    n = 6
    rng = np.random.default_rng(1)
    st = _euler_state_1d(n, rng)
    p = _oracle_1d(O.EULER, n, O.TRANSMISSIVE)
    ax, _ = O.alpha(p, st)
    L, _ = O.rhs(p, st, ax)

    def zero_ghost(a):
        out = np.pad(a, ((0, 0), (2, 2)), mode="edge")
        out[:, :2] = 0.0
        out[:, -2:] = 0.0
        return out

    Lz, _ = B.rhs_1d(B.euler_flux, st, p.dx, ax, p.gamma_lin, p.eps, O.TRANSMISSIVE,
                     pad_derivative=zero_ghost)
    assert _scale_err(L, Lz) > 1e-6


# ------------------------------------------------------- per-stage speeds

@pytest.mark.parametrize("per_stage", [0, 1])
@pytest.mark.parametrize("dim", [1, 2])
def test_step_matches_bruteforce_with_each_stage_speed(dim, per_stage):
    rng = np.random.default_rng(40 + dim)
    if dim == 1:
        n = 7
        st = _euler_state_1d(n, rng)
        p = _oracle_1d(O.EULER, n, O.TRANSMISSIVE, alpha_stage=per_stage)
        rhs = lambda s, a: B.rhs_1d(B.euler_flux, s, p.dx, a[0], p.gamma_lin, p.eps,
                                    O.TRANSMISSIVE)
    else:
        n = 5
        st = _euler_state_2d(n, rng)
        p = O.Problem(dim=2, flux=O.EULER, nx=n, ny=n, bc_x=O.TRANSMISSIVE, bc_y=O.PERIODIC,
                      gauss_q=2, weights=O.W_BETA, alpha_stage=per_stage)
        rhs = lambda s, a: B.rhs_2d(B.euler_flux, s, p.dx, p.dy, a[0], a[1], p.gamma_lin,
                                    p.eps, False, 2, O.TRANSMISSIVE, O.PERIODIC)
    ax, ay = O.alpha(p, st)
    dt = O.dt(p, ax, ay, 0.5)
    a0 = B.speeds(B.euler_flux, st)
    alphas_of = (lambda k, s: B.speeds(B.euler_flux, s)) if per_stage else (lambda k, s: a0)
    want = B.ssprk3(rhs, st, dt, alphas_of)
    got = O.step(p, st, ax, ay, dt)
    assert _scale_err(got, want) < 1e-11
    # with the other choice of speeds the step differs beyond the bar
    other = (lambda k, s: a0) if per_stage else (lambda k, s: B.speeds(B.euler_flux, s))
    assert _scale_err(got, B.ssprk3(rhs, st, dt, other)) > 1e-9
