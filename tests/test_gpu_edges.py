"""Edge cases of the GPU path against the oracle: the smallest grids the
library accepts (4 cells per axis: every stencil reaches across the
boundary, one strip and one segment hold the whole problem), strips and
segments cut short, a batch mixing tiny and larger problems of every
boundary type, and constant states (the scheme's degenerate case: every
smoothness indicator is zero, the weights are the linear ones, and the
state must not move)."""
import numpy as np
import pytest

import oracle as O
from gpu_util import oproblem, natural_scales, scaled_err, within_conditioning, oracle_sensitivity
from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

pytestmark = pytest.mark.gpu

RNG = np.random.default_rng(21)


def _random_euler(dim, nx, ny=1, bc=(W.PERIODIC, W.PERIODIC)):
    spec = W.Spec(dim=dim, flux=W.EULER, nx=nx, ny=ny, xlo=0.0, xhi=nx / 16.0, ylo=0.0,
                  yhi=ny / 16.0, bc_x=bc[0], bc_y=bc[1] if dim == 2 else W.PERIODIC,
                  t_end=1.0, name=f"edge-{dim}d-{nx}x{ny}")
    st = np.zeros(spec.shape())
    shape = (ny, nx)
    rho = RNG.uniform(0.5, 1.5, shape)
    p = RNG.uniform(0.5, 1.5, shape)
    u = RNG.uniform(-0.5, 0.5, shape)
    if dim == 1:
        st[0, :, :, :] = W.conserved_1d(rho, u, p)
    else:
        st[0] = W.conserved_2d(rho, u, RNG.uniform(-0.5, 0.5, shape), p)
    st[1:] = 0.1 * RNG.normal(size=st[1:].shape)
    return spec, st


def _step_parity(spec, st, cfg):
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        dt = h.step(want_dt=True)[0]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    ax, ay = O.alpha(p, st)
    assert abs(dt - O.dt(p, ax, ay, cfg.cfl)) <= 1e-15 * dt
    fn = lambda s: O.step(p, s, ax, ay, dt)   # noqa: E731
    S = natural_scales(spec, st)
    ok, err, bar = within_conditioning(gpu, fn(st), S, oracle_sensitivity(fn, st, S), 1e-12)
    assert ok, (spec.name, err, bar)


@pytest.mark.parametrize("bc", [W.PERIODIC, W.TRANSMISSIVE, W.REFLECTIVE])
@pytest.mark.parametrize("charwise", [0, 1])
def test_smallest_1d_grid(bc, charwise):
    spec, st = _random_euler(1, 4, bc=(bc, bc))
    _step_parity(spec, st, hw.default_config(1, precision=hw.F64, characteristic=charwise))


@pytest.mark.parametrize("bc", [W.PERIODIC, W.TRANSMISSIVE, W.REFLECTIVE])
@pytest.mark.parametrize("charwise", [0, 1])
def test_smallest_2d_grid(bc, charwise):
    spec, st = _random_euler(2, 4, 4, bc=(bc, bc))
    _step_parity(spec, st, hw.default_config(2, precision=hw.F64, gauss_q=2,
                                             characteristic=charwise))


@pytest.mark.parametrize("nx,ny", [(61, 9), (59, 33), (121, 65), (5, 130)])
def test_strips_and_segments_cut_short(nx, ny):
    """sizes around the 60 output columns of a strip and the 32 rows of a
    segment, mixed boundary types"""
    spec, st = _random_euler(2, nx, ny, bc=(W.TRANSMISSIVE, W.REFLECTIVE))
    _step_parity(spec, st, hw.default_config(2, precision=hw.F64, gauss_q=3))


def test_batch_of_tiny_and_larger_problems():
    specs, states = [], []
    for i, (nx, ny) in enumerate([(4, 4), (64, 4), (4, 70), (37, 29), (130, 61)]):
        bc = [(W.PERIODIC, W.PERIODIC), (W.TRANSMISSIVE, W.PERIODIC),
              (W.REFLECTIVE, W.TRANSMISSIVE), (W.REFLECTIVE, W.REFLECTIVE),
              (W.PERIODIC, W.REFLECTIVE)][i]
        s, st = _random_euler(2, nx, ny, bc=bc)
        s = W.Spec(dim=2, flux=W.EULER, nx=nx, ny=ny, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0,
                   bc_x=bc[0], bc_y=bc[1], t_end=1.0, name=f"batch-{i}")
        specs.append(s)
        states.append(st)
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2)
    with hw.Handle(specs, cfg) as h:
        for i, st in enumerate(states):
            h.set_state(i, st)
        dts = h.step(want_dt=True)
        outs = [h.get_state(i)[0] for i in range(len(specs))]
    for spec, st, dt, g in zip(specs, states, dts, outs):
        p = oproblem(spec, cfg)
        ax, ay = O.alpha(p, st)
        assert abs(dt - O.dt(p, ax, ay, cfg.cfl)) <= 1e-15 * dt
        fn = lambda s: O.step(p, s, ax, ay, dt)   # noqa: E731
        S = natural_scales(spec, st)
        ok, err, bar = within_conditioning(g, fn(st), S, oracle_sensitivity(fn, st, S), 1e-12)
        assert ok, (spec.name, err, bar)


@pytest.mark.parametrize("prec", [hw.F64, hw.F32, hw.F32_ACC64, hw.F32_KAHAN])
@pytest.mark.parametrize("charwise", [0, 1])
def test_constant_state_does_not_move(prec, charwise):
    """A uniform flow with zero derivative means: every flux difference and
    every derivative update vanishes up to the rounding of the RK
    combination (cell averages exactly representable in each precision)."""
    n = 70
    spec = W.Spec(dim=2, flux=W.EULER, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0,
                  bc_x=W.PERIODIC, bc_y=W.TRANSMISSIVE, t_end=1.0, name="uniform")
    st = np.zeros(spec.shape())
    U = W.conserved_2d(1.0, 0.5, -0.25, 1.0)
    for c in range(4):
        st[0, c] = U[c]
    cfg = hw.default_config(2, precision=prec, gauss_q=2, characteristic=charwise)
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        for _ in range(4):
            h.step()
        gpu, t = h.get_state(0)
    tol = 1e-14 if prec in (hw.F64, hw.F32_ACC64, hw.F32_KAHAN) else 1e-6
    for c in range(4):
        assert np.abs(gpu[0, c] - U[c]).max() <= tol * max(abs(U[c]), 1.0), (c, prec)
    assert np.abs(gpu[1:]).max() <= (1e-12 if tol < 1e-10 else 1e-5)
    assert t > 0
