"""GPU parity of the reconstruction in local characteristic variables (1D
Euler; remark closing Sec. 2.2) against the oracle, on the shock tubes of
Sec. 3.2 and uneven batches.  Bars as for the component-wise path: FP64
1e-12 per operator and step against natural scales, 1e-10 on whole runs;
FP32 bulk 2e-5 in relative L1 of the averages."""
import numpy as np
import pytest

import oracle as O
from gpu_util import (oproblem, l1_rel, natural_scales, scaled_err, rhs_scales,
                      oracle_sensitivity, within_conditioning)
from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

pytestmark = pytest.mark.gpu

CASES = {
    "lax-400": lambda: W.lax_1d(400),
    "shu-osher-777": lambda: W.shu_osher_1d(777),
    "riemann-600": lambda: W.riemann_1d(3, nx=600),
    "euler-smooth-257": lambda: W.euler_1d_smooth(257),
}


def _cfg(prec=hw.F64, **kw):
    return hw.default_config(1, precision=prec, characteristic=1, **kw)


@pytest.mark.parametrize("case", list(CASES))
def test_charwise_rhs_and_step_f64(case):
    spec, st = CASES[case]()
    cfg = _cfg()
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        ax, _ = h.alpha(0)
        L, Uh = h.rhs(0)
        dt = h.step(want_dt=True)[0]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    assert p.charwise == 1
    Lr, Uhr = O.rhs(p, st, ax, 0.0)
    S = natural_scales(spec, st)
    assert scaled_err(Uh, Uhr, S) < 1e-12, scaled_err(Uh, Uhr, S)
    assert scaled_err(L, Lr, rhs_scales(spec, st, ax, 0.0)) < 1e-12
    ref = O.step(p, st, ax, 0.0, dt)
    assert scaled_err(gpu, ref, S) < 1e-12, scaled_err(gpu, ref, S)
    # the projection is not a no-op on these data
    p0 = oproblem(spec, hw.default_config(1, precision=hw.F64))
    if case != "euler-smooth-257":
        assert scaled_err(O.rhs(p0, st, ax, 0.0)[0], Lr, rhs_scales(spec, st, ax, 0.0)) > 1e-6


def test_charwise_lax_run_to_final_time():
    """Lax problem, N = 400, CFL 0.6 to T = 0.16: same step count; the final
    state is held to the conditioning-aware bar of the long runs (1e-15
    relative input perturbations move the oracle's own final state by ~1e-6
    in mean: the unlimited scheme amplifies rounding behind the shock)."""
    spec, st = W.lax_1d(400)
    cfg = _cfg()
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        steps = h.run_to_time()
        gpu, t = h.get_state(0)
    p = oproblem(spec, cfg)
    ref, n = O.run(p, st, 0.0, 0.16, cfg.cfl)
    assert steps == n and t == 0.16
    S = natural_scales(spec, st)
    sens = oracle_sensitivity(lambda s: O.run(p, s, 0.0, 0.16, cfg.cfl)[0], st, S)
    ok, err, bar = within_conditioning(gpu, ref, S, sens, 1e-10)
    assert ok, (err, bar)


@pytest.mark.parametrize("prec", [hw.F32, hw.F32_ACC64, hw.F32_KAHAN])
def test_charwise_reduced_precision(prec):
    spec, st = W.lax_1d(400)
    cfg = _cfg(prec)
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        dts = [h.step(want_dt=True)[0] for _ in range(5)]
        gpu, _ = h.get_state(0)
    p = oproblem(spec, cfg)
    ref = st
    for dt in dts:
        ax, _ = O.alpha(p, ref)
        ref = O.step(p, ref, ax, 0.0, dt)
    assert l1_rel(gpu[0], ref[0]) < 2e-5, l1_rel(gpu[0], ref[0])


def test_charwise_batched_uneven_problems():
    entries = W.batched_1d(seed=4, nprob=7, nmin=40, nmax=900, t_end=0.01)
    specs = [e[0] for e in entries]
    states = [W.batched_1d_state(e) for e in entries]
    cfg = _cfg()
    with hw.Handle(specs, cfg) as h:
        for i, s in enumerate(states):
            h.set_state(i, s)
        steps = h.run_to_time()
        outs = [h.get_state(i) for i in range(len(specs))]
    nmax = 0
    for spec, s, (g, t) in zip(specs, states, outs):
        p = oproblem(spec, cfg)
        ref, n = O.run(p, s, 0.0, 0.01, cfg.cfl)
        nmax = max(nmax, n)
        assert t == 0.01
        assert scaled_err(g, ref, natural_scales(spec, s)) < 1e-10
    assert steps == nmax


def test_charwise_2d_is_rejected_for_now():
    spec, st = W.quadrant_vortex_2d(16, seed=3)
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2, characteristic=1)
    with pytest.raises(hw.HwenoError):
        hw.Handle([spec], cfg)
