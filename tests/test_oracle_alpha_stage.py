"""Pins of the oracle's per-stage Lax-Friedrichs speeds (the option in
which stages 2 and 3 take alpha from their own input states U^(1), U^(2)
instead of U^n; the time step always comes from U^n).  The step is checked
against its definition composed from the operator: U1 = Uhat^n + dt L(U^n),
U2 = 3/4 Uhat^n + 1/4 (Uhat1 + dt L(U1)), U^(n+1) = 1/3 Uhat^n + 2/3 (Uhat2 +
dt L(U2)), each L and Uhat evaluated with the speeds the option selects."""
import numpy as np
import pytest

import oracle as O
from paper_2607_24325_amd import workloads as W


def _problem(spec, **kw):
    d = dict(dim=spec.dim, flux=spec.flux, nx=spec.nx, ny=spec.ny, xlo=spec.xlo, xhi=spec.xhi,
             ylo=spec.ylo, yhi=spec.yhi, bc_x=spec.bc_x, bc_y=spec.bc_y, adv=spec.adv,
             gauss_q=2, weights=O.W_BETA)
    d.update(kw)
    return O.Problem(**d)


def _composed(p, st, dt, per_stage):
    a0 = O.alpha(p, st)
    L0, H0 = O.rhs(p, st, *a0)
    u1 = H0 + dt * L0
    a1 = O.alpha(p, u1) if per_stage else a0
    L1, H1 = O.rhs(p, u1, *a1)
    u2 = 0.75 * H0 + 0.25 * (H1 + dt * L1)
    a2 = O.alpha(p, u2) if per_stage else a0
    L2, H2 = O.rhs(p, u2, *a2)
    return H0 / 3.0 + 2.0 / 3.0 * (H2 + dt * L2), (a0, a1, a2)


CASES = {
    "riemann-1d": lambda: W.riemann_1d(4, nx=80),
    "blast-1d": lambda: W.blast_1d(60),
    "quadrant-vortex-2d": lambda: W.quadrant_vortex_2d(20, seed=5),
}


@pytest.mark.parametrize("per_stage", [0, 1])
@pytest.mark.parametrize("case", list(CASES))
def test_step_equals_its_composition(case, per_stage):
    spec, st = CASES[case]()
    p = _problem(spec, alpha_stage=per_stage)
    ax, ay = O.alpha(p, st)
    dt = O.dt(p, ax, ay, 0.6)
    got = O.step(p, st, ax, ay, dt)
    want, alphas = _composed(p, st, dt, per_stage)
    scale = np.abs(want).max(axis=tuple(range(2, want.ndim)), keepdims=True) + 1e-300
    assert (np.abs(got - want) / scale).max() < 1e-13
    if per_stage:   # the option does change the speeds on these data
        assert alphas[1] != alphas[0] and alphas[2] != alphas[0]
        p0 = _problem(spec)
        assert np.abs(O.step(p0, st, ax, ay, dt) - got).max() > 0


def test_constant_speed_laws_are_unaffected():
    spec, st = W.advection_2d(24)
    p0 = _problem(spec)
    p1 = _problem(spec, alpha_stage=1)
    ax, ay = O.alpha(p0, st)
    np.testing.assert_array_equal(O.step(p0, st, ax, ay, 1e-3), O.step(p1, st, ax, ay, 1e-3))


def test_window_stepping_is_refused():
    spec, st = W.quadrant_vortex_2d(20, seed=5)
    p = _problem(spec, alpha_stage=1)
    ax, ay = O.alpha(p, st)
    with pytest.raises(O.OracleError):
        O.step_window(p, st, ax, ay, 1e-3, 0, 0, 3, 3)
