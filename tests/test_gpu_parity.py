"""GPU parity: the HIP path, called through the C ABI, against the FP64 CPU
oracle on the same seeded inputs (element by element).

FP64 bar: 1e-12 relative, per operator evaluation and per step, each
(variable, component) plane measured against its natural scale (see
gpu_util.natural_scales; L against the state scale times alpha/dx).
Results that only differ in the order of the IEEE operations stay far below.
"""
import numpy as np
import pytest

import oracle as O
from gpu_util import (l1_rel, l1_scaled, natural_scales, oproblem, plane_rel, rhs_scales,
                      scaled_err)
from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

pytestmark = pytest.mark.gpu

F64_TOL = 1e-12


def _one(spec, st, cfg):
    h = hw.Handle([spec], cfg)
    h.set_state(0, st)
    return h


# ------------------------------------------------------------- operators --

CASES_2D = {
    "euler-quadrant-vortex-96": lambda: W.quadrant_vortex_2d(96, seed=7),
    "euler-quadrant-vortex-130x70-transmissive": lambda: _nonsquare(),
    "euler-smooth-40": lambda: W.euler_2d_smooth(40),
    "burgers-40": lambda: W.burgers_2d(40),
    "advection-37": lambda: W.advection_2d(37),
}


def _nonsquare():
    spec, _ = W.quadrant_vortex_2d(4, seed=1)
    spec = W.Spec(dim=2, flux=W.EULER, nx=130, ny=70, xlo=0, xhi=1.3, ylo=0, yhi=0.7,
                  bc_x=W.TRANSMISSIVE, bc_y=W.PERIODIC, t_end=0.1, name="nonsquare")
    rng = np.random.default_rng(5)
    J, I = np.meshgrid(np.arange(70), np.arange(130), indexing="ij")
    rho = 0.5 + 0.3 * (I > 60) + 0.1 * np.sin(0.2 * I + 0.3 * J)
    u = 0.3 * np.cos(0.1 * J)
    v = -0.2 + 0.1 * (J > 40)
    p = 0.7 + 0.2 * (I + J > 90)
    st = np.zeros(spec.shape())
    st[0] = W.conserved_2d(rho, u, v, p)
    st[1] = 0.05 * rng.normal(size=st[1].shape)
    st[2] = 0.05 * rng.normal(size=st[2].shape)
    return spec, st


@pytest.mark.parametrize("Q", [2, 3])
@pytest.mark.parametrize("case", list(CASES_2D))
def test_2d_rhs_f64(case, Q):
    spec, st = CASES_2D[case]()
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=Q)
    with _one(spec, st, cfg) as h:
        ax, ay = h.alpha(0)
        L, Uh = h.rhs(0)
    p = oproblem(spec, cfg)
    oax, oay = O.alpha(p, st)
    assert abs(ax - oax) <= 1e-15 * oax and abs(ay - oay) <= 1e-15 * max(oay, 1e-300)
    Lr, Uhr = O.rhs(p, st, ax, ay)
    S = natural_scales(spec, st)
    assert scaled_err(Uh, Uhr, S) < F64_TOL, scaled_err(Uh, Uhr, S)
    assert scaled_err(L, Lr, rhs_scales(spec, st, ax, ay)) < F64_TOL


@pytest.mark.parametrize("case", list(CASES_2D))
def test_2d_step_f64(case):
    spec, st = CASES_2D[case]()
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2)
    with _one(spec, st, cfg) as h:
        dt = h.step(want_dt=True)[0]
        gpu, t = h.get_state(0)
    p = oproblem(spec, cfg)
    ax, ay = O.alpha(p, st)
    assert abs(dt - O.dt(p, ax, ay, cfg.cfl)) <= 1e-14 * dt
    ref = O.step(p, st, ax, ay, dt)
    err = scaled_err(gpu, ref, natural_scales(spec, st))
    assert err < F64_TOL, err
    assert t == dt


CASES_1D = {
    "riemann-600": lambda: W.riemann_1d(3, nx=600),
    "euler-smooth-257": lambda: W.euler_1d_smooth(257),
    "burgers-100": lambda: W.burgers_1d(100),
    "advection-200": lambda: W.advection_1d(200),
}


@pytest.mark.parametrize("case", list(CASES_1D))
def test_1d_rhs_and_step_f64(case):
    spec, st = CASES_1D[case]()
    cfg = hw.default_config(1, precision=hw.F64)
    with _one(spec, st, cfg) as h:
        ax, _ = h.alpha(0)
        L, Uh = h.rhs(0)
        dt = h.step(want_dt=True)[0]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    Lr, Uhr = O.rhs(p, st, ax, 0.0)
    S = natural_scales(spec, st)
    assert scaled_err(Uh, Uhr, S) < F64_TOL, scaled_err(Uh, Uhr, S)
    assert scaled_err(L, Lr, rhs_scales(spec, st, ax, 0.0)) < F64_TOL
    ref = O.step(p, st, ax, 0.0, dt)
    assert scaled_err(gpu, ref, S) < F64_TOL, scaled_err(gpu, ref, S)


def test_1d_advection_headline_run_to_time():
    """u_t + u_x = 0, N = 200, gamma = (0.98, 0.01, 0.01), CFL 0.6 to t = 2:
    step count and final state match the oracle (L1 <= 1e-10)."""
    spec, st = W.advection_1d(200)
    cfg = hw.default_config(1, precision=hw.F64, gamma_lin=(0.98, 0.01, 0.01))
    with _one(spec, st, cfg) as h:
        steps = h.run_to_time()
        gpu, t = h.get_state(0)
    p = oproblem(spec, cfg)
    ref, n = O.run(p, st, 0.0, 2.0, 0.6)
    assert steps == n == 334 and t == 2.0
    assert np.abs(gpu[0] - ref[0]).mean() <= 1e-10
    assert scaled_err(gpu, ref, natural_scales(spec, st)) < 1e-10


# ------------------------------------------------------ reduced precision --

@pytest.mark.parametrize("prec,tol", [(hw.F32, 2e-5), (hw.F32_ACC64, 2e-5), (hw.F32_KAHAN, 2e-5)])
def test_2d_euler_step_reduced_precision(prec, tol):
    spec, st = W.quadrant_vortex_2d(96, seed=7)
    cfg = hw.default_config(2, precision=prec, gauss_q=2)
    with _one(spec, st, cfg) as h:
        dts = [h.step(want_dt=True)[0] for _ in range(3)]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    ref = st
    for dt in dts:
        ax, ay = O.alpha(p, ref)
        ref = O.step(p, ref, ax, ay, dt)
    assert l1_rel(gpu[0], ref[0]) < tol, l1_rel(gpu[0], ref[0])
    # every plane, the derivative averages included, in its natural scale
    S = natural_scales(spec, st)
    print(f"2D 96^2 three steps prec {prec}: L1 {l1_scaled(gpu, ref, S):.3e} "
          f"max {scaled_err(gpu, ref, S):.3e}", flush=True)
    assert l1_scaled(gpu, ref, S) < tol
    assert scaled_err(gpu, ref, S) < 20 * tol


@pytest.mark.parametrize("prec", [hw.F32, hw.F32_ACC64, hw.F32_KAHAN])
def test_1d_euler_step_reduced_precision(prec):
    spec, st = W.riemann_1d(3, nx=600)
    cfg = hw.default_config(1, precision=prec)
    with _one(spec, st, cfg) as h:
        dts = [h.step(want_dt=True)[0] for _ in range(5)]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    ref = st
    for dt in dts:
        ax, _ = O.alpha(p, ref)
        ref = O.step(p, ref, ax, 0.0, dt)
    assert l1_rel(gpu[0], ref[0]) < 2e-5
    S = natural_scales(spec, st)
    print(f"1D 600 five steps prec {prec}: L1 {l1_scaled(gpu, ref, S):.3e} "
          f"max {scaled_err(gpu, ref, S):.3e}", flush=True)
    assert l1_scaled(gpu, ref, S) < 2e-5
    assert scaled_err(gpu, ref, S) < 4e-4


@pytest.mark.parametrize("prec", [hw.F32_ACC64, hw.F32_KAHAN])
def test_mixed_precision_conserves_cell_average_totals(prec):
    """FP32 reconstruction with FP64 (or compensated FP32) flux differences and
    cell averages: the periodic totals stay fixed to ~double rounding."""
    spec, st = W.euler_2d_smooth(64)
    cfg = hw.default_config(2, precision=prec, gauss_q=2)
    with _one(spec, st, cfg) as h:
        for _ in range(5):
            h.step()
        gpu, _ = h.get_state(0)
    tot0 = st[0].sum(axis=(1, 2))
    tot = gpu[0].sum(axis=(1, 2))
    assert np.all(np.abs(tot - tot0) <= 1e-12 * np.abs(tot0))


# ------------------------------------------------ tiling and determinism --

@pytest.mark.parametrize("prec", [hw.F64, hw.F32_ACC64])
def test_results_independent_of_tiling_and_graphs(prec):
    """Bitwise-identical results for every segment height, persistent grid
    size, register variant and graph/eager launch: no races, no order
    dependence."""
    spec, st = W.quadrant_vortex_2d(128, seed=2)
    cfg = hw.default_config(2, precision=prec, gauss_q=2)
    outs = []
    for rows, grid, graph, var in [(64, 0, 1, 0), (16, 0, 1, 0), (128, 0, 0, 0), (32, 37, 1, 0),
                                   (8, 256, 0, 0), (32, 0, 1, 1), (24, 512, 1, 1), (48, 0, 0, 1)]:
        with _one(spec, st, cfg) as h:
            h.set_tuning(tile_rows=rows, grid_blocks=grid, use_graph=graph, variant=var)
            for _ in range(3):
                h.step()
            outs.append(h.get_state(0)[0])
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


@pytest.mark.parametrize("prec", [hw.F32_ACC64, hw.F32_KAHAN, hw.F32, hw.F64])
def test_1d_results_and_time_steps_independent_of_launch(prec):
    """1D: bitwise-identical states after three steps for one workgroup per
    tile or a persistent grid, graph or eager launch (and the register
    variant setting, which the 1D kernels ignore); every time step equals
    the one the oracle's speeds of the state give."""
    entries = W.batched_1d(seed=5, nprob=12, nmin=40, nmax=700)
    specs = [e[0] for e in entries]
    states = [W.batched_1d_state(e) for e in entries]
    cfg = hw.default_config(1, precision=prec)
    outs = []
    for grid, graph, var in [(0, 1, 0), (0, 1, 1), (5, 0, 1), (3, 1, 0), (0, 0, 1)]:
        with hw.Handle(specs, cfg) as h:
            for i, s in enumerate(states):
                h.set_state(i, s)
            h.set_tuning(grid_blocks=grid, use_graph=graph, variant=var)
            h.step()
            for _ in range(2):
                cur = [h.get_state(i)[0] for i in range(len(specs))]
                dts = h.step(want_dt=True)
                for i, sp in enumerate(specs):
                    p = oproblem(sp, cfg)
                    ax, ay = O.alpha(p, cur[i])
                    assert dts[i] == O.dt(p, ax, ay, cfg.cfl), (grid, graph, var, i)
            outs.append([h.get_state(i)[0] for i in range(len(specs))])
    for o in outs[1:]:
        for a, b in zip(o, outs[0]):
            np.testing.assert_array_equal(a, b)


@pytest.mark.parametrize("prec", [hw.F32_ACC64, hw.F64, hw.F32_KAHAN])
def test_fused_wave_speeds_equal_a_fresh_reduction(prec):
    """Stage 3 gathers the wave speeds of the state it writes (in groups of
    rows, one wave per row of a group); the next step's time step must be
    exactly the one that the speeds of that state give.  Segment heights
    that leave partial groups and a last short segment are included."""
    spec, st = _nonsquare()
    cfg = hw.default_config(2, precision=prec, gauss_q=2)
    p = oproblem(spec, cfg)
    for rows in (8, 13, 32, 64):
        with _one(spec, st, cfg) as h:
            h.set_tuning(tile_rows=rows)
            h.step()
            for _ in range(3):
                cur, _ = h.get_state(0)
                ax, ay = O.alpha(p, cur)
                dt = h.step(want_dt=True)[0]
                assert dt == O.dt(p, ax, ay, cfg.cfl), (rows, dt, O.dt(p, ax, ay, cfg.cfl))


# -------------------------------------------------------------- batching --

def test_batched_2d_uneven_problems():
    entries = W.batched_2d(seed=11, nprob=5, nmin=20, nmax=140)
    specs = [e[0] for e in entries]
    states = [W.batched_2d_state(e) for e in entries]
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2)
    with hw.Handle(specs, cfg) as h:
        for i, s in enumerate(states):
            h.set_state(i, s)
        dts = h.step(want_dt=True)
        outs = [h.get_state(i)[0] for i in range(len(specs))]
    for spec, s, dt, g in zip(specs, states, dts, outs):
        p = oproblem(spec, cfg)
        ax, ay = O.alpha(p, s)
        assert abs(dt - O.dt(p, ax, ay, cfg.cfl)) <= 1e-14 * dt
        assert scaled_err(g, O.step(p, s, ax, ay, dt), natural_scales(spec, s)) < F64_TOL


def test_batched_1d_uneven_problems_run_to_time():
    entries = W.batched_1d(seed=1, nprob=6, nmin=40, nmax=700, t_end=0.02)
    specs = [e[0] for e in entries]
    states = [W.batched_1d_state(e) for e in entries]
    cfg = hw.default_config(1, precision=hw.F64)
    with hw.Handle(specs, cfg) as h:
        for i, s in enumerate(states):
            h.set_state(i, s)
        steps = h.run_to_time()
        outs = [h.get_state(i) for i in range(len(specs))]
    nmax = 0
    for spec, s, (g, t) in zip(specs, states, outs):
        p = oproblem(spec, cfg)
        ref, n = O.run(p, s, 0.0, 0.02, cfg.cfl)
        nmax = max(nmax, n)
        assert t == 0.02
        assert scaled_err(g, ref, natural_scales(spec, s)) < 1e-10
    assert steps == nmax


# ----------------------------------------------------------------- errors --

def test_nonadmissible_state_is_reported():
    spec, st = W.riemann_1d(3, nx=300)
    bad = st.copy()
    bad[0, 0, 0, 123] = -0.5   # negative density
    cfg = hw.default_config(1, precision=hw.F64)
    with _one(spec, bad, cfg) as h:
        h.step()
        with pytest.raises(hw.HwenoError) as ei:
            h.sync()
        assert ei.value.code == hw.ERR_NONFINITE and "i=123" in str(ei.value)
        with pytest.raises(hw.HwenoError):
            h.get_state(0)


def test_nonadmissible_state_reached_by_the_scheme_matches_oracle():
    """Problem 1390 of the seeded 4096-problem 1D batch (four Riemann states)
    develops a non-admissible state after 74 steps (the scheme has no
    positivity limiter): the GPU reports the same step and cell as the
    oracle, and the same time to within the problem's conditioning.  On the
    way to vacuum the sound speed comes from the cancellation in
    p = (gamma - 1)(E - rho |u|^2 / 2), so the time steps are ill-conditioned:
    a relative change of 1e-15 in the initial state moves the oracle's own
    time of failure by about 1.2e-12 relative.  The bar is the larger of
    1e-12 and 10x that change (the rule of the final-time tests)."""
    entries = W.batched_1d(seed=1, nprob=4096)
    spec, st = entries[1390][0], W.batched_1d_state(entries[1390])
    cfg = hw.default_config(1, precision=hw.F64)
    p = oproblem(spec, cfg)

    def oracle_failure(state):
        cur, t, n = state, 0.0, 0
        while True:
            try:
                ax, _ = O.alpha(p, cur)
            except O.OracleError as e:
                return t, n, int(str(e).split()[-1])
            dt = O.dt(p, ax, 0.0, cfg.cfl)
            cur = O.step(p, cur, ax, 0.0, dt)
            t += dt
            n += 1

    t, n, cell = oracle_failure(st)
    own = max(abs(oracle_failure(st * (1.0 + e))[0] - t) for e in (1e-15, -1e-15))
    tol = max(1e-12 * t, 10.0 * own)
    with _one(spec, st, cfg) as h:
        with pytest.raises(hw.HwenoError) as ei:
            h.run_to_time()
        assert ei.value.code == hw.ERR_NONFINITE
        assert f"i={cell} " in str(ei.value)
        t_gpu = float(str(ei.value).split("t=")[-1])
        print(f"t {t_gpu!r} (oracle {t!r}, relative {abs(t_gpu - t) / t:.3e}; "
              f"oracle's own change {own / t:.3e})")
        assert abs(t_gpu - t) <= tol
        assert n == 74
