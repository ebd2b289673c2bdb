"""Batched workloads at their real shapes, one launch per RK stage over all
problems, checked against the oracle on sampled problems.

* 4096 independent 1D Euler problems, N ~ U{256..8192} (seed 1): one step
  of every problem element by element, then a run to t = 0.05 with
  per-problem dt checked on 16 sampled problems.
* 256 independent 2D Euler problems, side ~ U{128..1024} (seed 11), mixed
  boundaries; two steps; 16 sampled problems against the oracle.
A problem whose state becomes non-admissible (no positivity limiter exists in
the scheme) must be reported as such by both sides.
"""
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np
import pytest

import oracle as O
from gpu_util import oproblem, natural_scales, scaled_err, l1_rel
from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

pytestmark = pytest.mark.gpu

T1 = 0.05


@pytest.fixture(scope="module")
def batch1d():
    entries = W.batched_1d(seed=1, nprob=4096, t_end=T1)
    return entries, [W.batched_1d_state(e) for e in entries]


def _oracle_run(args):
    """oracle run to t_end, and the same run from an input perturbed at the
    rounding level of the path under test (relative noise `pert`)"""
    spec, st, cfg, pert = args
    p = oproblem(spec, cfg)
    rng = np.random.default_rng(spec.nx)
    try:
        out, n = O.run(p, st, 0.0, spec.t_end, cfg.cfl)
        out2, _ = O.run(p, st * (1.0 + pert * rng.standard_normal(st.shape)), 0.0,
                        spec.t_end, cfg.cfl)
        return out, out2, n, None
    except O.OracleError as e:
        return None, None, None, str(e)


def _oracle_step(args):
    spec, st, cfg, dt = args
    p = oproblem(spec, cfg)
    ax, _ = O.alpha(p, st)
    return O.step(p, st, ax, 0.0, dt)


@pytest.mark.parametrize("prec", [hw.F64, hw.F32_ACC64])
def test_batched_1d_4096_problems(batch1d, prec):
    """One step of all 4096 problems element by element (FP64: 1e-12 of the
    scale; FP32 bulk: 2e-5, set by the single-precision cancellation in the
    derivative fluxes at contacts, where dp = (gamma-1)(dE - u dm + ...) is
    a small difference of terms of size |jump|/dx), then the run to t = 0.05 on 16 sampled problems.
    Behind strong shocks the scheme amplifies rounding-level differences
    (no limiter, component-wise reconstruction): a 1e-15 relative input
    perturbation moves the oracle's own t = 0.05 state by up to ~1e-2 of the
    scale.  The run is therefore held to a conditioning-aware bar: its
    distance from the oracle may be at most a few times the distance between
    two oracle runs whose inputs differ at the path's rounding level (1e-15
    for FP64, 1e-7 for FP32 bulk), and never more than 1e-10 (FP64) or 2e-5
    (FP32 bulk, density L1) where the oracle is insensitive."""
    entries, states = batch1d
    specs = [e[0] for e in entries]
    cfg = hw.default_config(1, precision=prec)
    sample = list(range(0, len(specs), len(specs) // 16))
    with hw.Handle(specs, cfg) as h:
        for i, st in enumerate(states):
            h.set_state(i, st)
        dts = h.step(want_dt=True)
        one = [h.get_state(i)[0] for i in range(len(specs))]
        for i, st in enumerate(states):
            h.set_state(i, st)
        try:
            h.run_to_time()
        except hw.HwenoError:
            pass
        gpu = {}
        for i in sample:
            try:
                gpu[i] = h.get_state(i)
            except hw.HwenoError as e:
                gpu[i] = e
    O.set_threads(1)
    workers = min(16, os.cpu_count() or 1)
    with ThreadPoolExecutor(max_workers=workers) as ex:
        ref1 = list(ex.map(_oracle_step, [(specs[i], states[i], cfg, dts[i])
                                          for i in range(len(specs))]))
    step_tol = 1e-12 if prec == hw.F64 else 2e-5
    for i in range(len(specs)):
        err = scaled_err(one[i], ref1[i], natural_scales(specs[i], states[i]))
        assert err < step_tol, (i, err)
    pert = 1e-15 if prec == hw.F64 else 1e-7
    with ThreadPoolExecutor(max_workers=workers) as ex:
        refs = list(ex.map(_oracle_run, [(specs[i], states[i], cfg, pert) for i in sample]))
    O.set_threads(0)
    n_checked = 0
    for i, (ref, ref2, n, err) in zip(sample, refs):
        g = gpu[i]
        if err is not None:   # the oracle finds the state non-admissible: so must the GPU
            assert isinstance(g, hw.HwenoError) and g.code == hw.ERR_NONFINITE, (i, err)
            continue
        assert not isinstance(g, hw.HwenoError), (i, str(g))
        out, t = g
        assert t == T1
        if prec == hw.F64:
            S = natural_scales(specs[i], states[i])
            bar = max(1e-10, 10.0 * scaled_err(ref2, ref, S))
            assert scaled_err(out, ref, S) <= bar, (i, scaled_err(out, ref, S), bar)
        else:
            bar = max(2e-5, 10.0 * l1_rel(ref2[0], ref[0]))
            assert l1_rel(out[0], ref[0]) <= bar, (i, l1_rel(out[0], ref[0]), bar)
        n_checked += 1
    assert n_checked >= 12


@pytest.mark.parametrize("prec,tol", [(hw.F64, 1e-12), (hw.F32_ACC64, 2e-5), (hw.F32_KAHAN, 2e-5)])
def test_batched_2d_256_problems(prec, tol):
    entries = W.batched_2d(seed=11, nprob=256)
    specs = [e[0] for e in entries]
    cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5)
    sample = list(range(0, 256, 16))
    init = {}
    with hw.Handle(specs, cfg) as h:
        for i, e in enumerate(entries):
            st = W.batched_2d_state(e)
            if i in sample:
                init[i] = st
            h.set_state(i, st)
        dts = [h.step(want_dt=True) for _ in range(2)]
        outs = {i: h.get_state(i)[0] for i in sample}
    O.set_threads(os.cpu_count() or 1)
    for i in sample:
        p = oproblem(specs[i], cfg)
        ref = init[i]
        for d in dts:
            ax, ay = O.alpha(p, ref)
            assert abs(d[i] - O.dt(p, ax, ay, cfg.cfl)) <= (1e-14 if prec == hw.F64 else 1e-5) * d[i]
            ref = O.step(p, ref, ax, ay, d[i])
        err = scaled_err(outs[i], ref, natural_scales(specs[i], init[i]))
        assert err < tol, (i, specs[i].nx, err)
