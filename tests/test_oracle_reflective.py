"""Pins of the oracle's solid-wall (reflective) boundary, used by the blast
wave problem of Sec. 3.2.  A wall is equivalent to extending the data by
its mirror image: the normal momentum odd, every other conserved quantity
even, the derivative mean along the wall normal of opposite parity.  The
reflective run must therefore equal a periodic run on the mirror-doubled
domain, restricted to the original half -- a check that goes through the
periodic path only."""
import numpy as np
import pytest

import oracle as O
from paper_2607_24325_amd import workloads as W


def _mirror_x(st, dim):
    """mirror image across the right end of the domain in x (cells reversed)"""
    m = st[..., ::-1].copy()
    m[:, 1] *= -1.0     # normal (x) momentum odd
    m[1] *= -1.0        # x-derivative mean: opposite parity
    return m


def _mirror_y(st):
    m = st[:, :, ::-1, :].copy()
    m[:, 2] *= -1.0     # y momentum odd
    m[2] *= -1.0        # y-derivative mean
    return m


@pytest.mark.parametrize("charwise", [0, 1])
def test_1d_wall_equals_periodic_mirror_doubling(charwise):
    spec, st = W.blast_1d(60)
    n = spec.nx
    p = O.Problem(dim=1, flux=O.EULER, nx=n, xlo=0.0, xhi=1.0, bc_x=O.REFLECTIVE,
                  weights=O.W_BETA, charwise=charwise)
    d = np.concatenate([st, _mirror_x(st, 1)], axis=3)
    pd = O.Problem(dim=1, flux=O.EULER, nx=2 * n, xlo=0.0, xhi=2.0, bc_x=O.PERIODIC,
                   weights=O.W_BETA, charwise=charwise)
    ax, _ = O.alpha(p, st)
    assert ax == O.alpha(pd, d)[0]
    dt = O.dt(p, ax, 0.0, 0.6)
    a, b = st, d
    for _ in range(6):
        a = O.step(p, a, ax, 0.0, dt)
        b = O.step(pd, b, ax, 0.0, dt)
    scale = np.abs(a).max(axis=3, keepdims=True)
    assert (np.abs(a - b[..., :n]) / scale).max() < 1e-12
    assert (np.abs(_mirror_x(a, 1) - b[..., n:]) / scale).max() < 1e-12


def test_2d_walls_equal_periodic_mirror_doubling():
    spec, st = W.quadrant_vortex_2d(12, seed=4)
    n = spec.nx
    base = dict(dim=2, flux=O.EULER, gauss_q=2, weights=O.W_BETA)
    p = O.Problem(nx=n, ny=n, xlo=0, xhi=1, ylo=0, yhi=1, bc_x=O.REFLECTIVE,
                  bc_y=O.REFLECTIVE, **base)
    row = np.concatenate([st, _mirror_x(st, 2)], axis=3)
    d = np.concatenate([row, _mirror_y(row)], axis=2)
    pd = O.Problem(nx=2 * n, ny=2 * n, xlo=0, xhi=2, ylo=0, yhi=2, bc_x=O.PERIODIC,
                   bc_y=O.PERIODIC, **base)
    ax, ay = O.alpha(p, st)
    assert (ax, ay) == O.alpha(pd, d)
    dt = 0.5 * O.dt(p, ax, ay, 0.6)
    a = O.step(p, st, ax, ay, dt)
    b = O.step(pd, d, ax, ay, dt)
    scale = np.abs(a).max(axis=(2, 3), keepdims=True)
    assert (np.abs(a - b[:, :, :n, :n]) / scale).max() < 1e-12


def test_walls_conserve_mass_and_energy():
    """no flux of mass or energy through a wall: the totals stay fixed"""
    spec, st = W.blast_1d(200)
    p = O.Problem(dim=1, flux=O.EULER, nx=200, bc_x=O.REFLECTIVE, weights=O.W_BETA, charwise=1)
    out, steps = O.run(p, st, 0.0, 0.01, 0.6)
    t0 = st[0, :, 0].sum(axis=1)
    t1 = out[0, :, 0].sum(axis=1)
    assert steps > 100
    assert abs(t1[0] - t0[0]) <= 1e-13 * t0[0]
    assert abs(t1[2] - t0[2]) <= 1e-12 * t0[2]


def test_blast_wave_runs_to_final_time():
    """Sec. 3.2 blast wave, N = 400, CFL 0.6, T = 0.038 in characteristic
    variables: the run completes with positive density, and the peak of the
    collision region lies in the range known for this problem at this
    resolution (about 5-6.5)."""
    spec, st = W.blast_1d(400)
    p = O.Problem(dim=1, flux=O.EULER, nx=400, bc_x=O.REFLECTIVE, weights=O.W_BETA, charwise=1)
    out, _ = O.run(p, st, 0.0, 0.038, 0.6)
    rho = out[0, 0, 0]
    assert rho.min() > 0.1 and 5.0 < rho.max() < 6.5
    x = (np.arange(400) + 0.5) / 400
    assert 0.76 < x[np.argmax(rho)] < 0.82


def test_reflective_rejected_for_scalar_laws():
    spec, st = W.burgers_1d(16)
    p = O.Problem(dim=1, flux=O.BURGERS, nx=16, bc_x=O.REFLECTIVE)
    with pytest.raises(O.OracleError):
        O.rhs(p, st, 1.0)


@pytest.mark.parametrize("dim", [1, 2])
def test_window_step_at_walls_equals_full_step(dim):
    """Windows touching the walls (their margins refilled with the signed
    mirror images after each stage) reproduce the full-grid step."""
    if dim == 1:
        spec, st = W.blast_1d(48)
        p = O.Problem(dim=1, flux=O.EULER, nx=48, bc_x=O.REFLECTIVE, weights=O.W_BETA)
        win = [(0, 0, 3, 1), (45, 0, 3, 1), (20, 0, 4, 1)]
    else:
        spec, st = W.quadrant_vortex_2d(20, seed=6)
        p = O.Problem(dim=2, flux=O.EULER, nx=20, ny=20, bc_x=O.REFLECTIVE, bc_y=O.REFLECTIVE,
                      gauss_q=2, weights=O.W_BETA)
        win = [(0, 0, 3, 3), (17, 18, 3, 2), (0, 9, 2, 4), (8, 19, 4, 1)]
    ax, ay = O.alpha(p, st)
    dt = 0.5 * O.dt(p, ax, ay, 0.6)
    full = O.step(p, st, ax, ay, dt)
    for (i0, j0, wi, wj) in win:
        w = O.step_window(p, st, ax, ay, dt, i0, j0, wi, wj)
        np.testing.assert_array_equal(w, full[:, :, j0:j0 + w.shape[2], i0:i0 + wi])
