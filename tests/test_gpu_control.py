"""Step control on the GPU against the oracle: the wave speeds that the
Lax-Friedrichs flux and the CFL rule (Sec. 2.1, Sec. 3) use after a state is
set again on a handle that has already stepped, after an autotuning pass
(which times steps and restores the state it started from), and in the
lighter step the library launches once stage 3 has gathered the speeds of
the state it wrote (no reduction kernel, step counters set by the dt
kernel)."""
import numpy as np
import pytest

import oracle as O
from gpu_util import oproblem, natural_scales, scaled_err
from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

pytestmark = pytest.mark.gpu

CFL = 0.5


def _cfg():
    return hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=CFL)


def _oracle_steps(p, st, n):
    dts = []
    for _ in range(n):
        ax, ay = O.alpha(p, st)
        dt = O.dt(p, ax, ay, CFL)
        st = O.step(p, st, ax, ay, dt)
        dts.append(dt)
    return st, dts


@pytest.mark.parametrize("graph", [1, 0])
def test_set_state_again_after_steps(graph):
    """Problem 0 steps three times and is then given a state with other
    speeds: the next two steps follow the new state (dt from its own speeds,
    not from the speeds stage 3 gathered before); problem 1 keeps its own
    evolution over all five steps."""
    cfg = _cfg()
    spec0, sa = W.quadrant_vortex_2d(64, seed=3)
    _, sb = W.quadrant_vortex_2d(64, seed=4)
    spec1, sc = W.quadrant_vortex_2d(48, seed=5)
    with hw.Handle([spec0, spec1], cfg) as h:
        h.set_tuning(use_graph=graph)
        h.set_state(0, sa)
        h.set_state(1, sc)
        dts = [h.step(want_dt=True) for _ in range(3)]
        h.set_state(0, sb)
        dts += [h.step(want_dt=True) for _ in range(2)]
        g0, t0 = h.get_state(0)
        g1, t1 = h.get_state(1)
    p0, p1 = oproblem(spec0, cfg), oproblem(spec1, cfg)
    ref0, odt0 = _oracle_steps(p0, sb, 2)
    ref1, odt1 = _oracle_steps(p1, sc, 5)
    # the speeds of the old state would give another dt by a few percent
    _, stale = _oracle_steps(p0, sa, 4)
    assert abs(stale[3] - odt0[0]) > 1e-3 * odt0[0]
    for k in range(2):
        assert abs(dts[3 + k][0] - odt0[k]) <= 1e-14 * odt0[k], (k, dts[3 + k][0], odt0[k])
    for k in range(5):
        assert abs(dts[k][1] - odt1[k]) <= 1e-12 * odt1[k], (k, dts[k][1], odt1[k])
    assert abs(t0 - sum(odt0)) <= 1e-14 and abs(t1 - sum(odt1)) <= 1e-14
    assert scaled_err(g0, ref0, natural_scales(spec0, sb)) < 1e-12
    assert scaled_err(g1, ref1, natural_scales(spec1, sc)) < 1e-11


@pytest.mark.parametrize("steps_before", [0, 2])
def test_autotune_restores_state_and_speeds(steps_before):
    """Autotuning right after set_state (speeds not yet reduced) and after
    two steps (speeds gathered by stage 3): the steps that follow equal the
    oracle's from the state before the tuning."""
    cfg = _cfg()
    spec, st = W.quadrant_vortex_2d(96, seed=7)
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        for _ in range(steps_before):
            h.step()
        h.autotune()
        dts = [h.step(want_dt=True)[0] for _ in range(2)]
        g, t = h.get_state(0)
    ref, odt = _oracle_steps(oproblem(spec, cfg), st, steps_before + 2)
    for k in range(2):
        want = odt[steps_before + k]
        assert abs(dts[k] - want) <= 1e-12 * want, (k, dts[k], want)
    assert abs(t - sum(odt)) <= 1e-13
    assert scaled_err(g, ref, natural_scales(spec, st)) < 1e-11


def test_autotune_cache_and_eager_mode(tmp_path, monkeypatch):
    """The tuner keeps the caller's eager mode in every candidate (and picks
    one of the configurations hweno_tuning_candidates lists), stores its
    winner in the cache file named by HWENO_TUNING_CACHE, and a second
    handle of the same class takes the stored configuration without timing;
    the tuned and cached runs give the bits of the default run."""
    cache = tmp_path / "tuning.jsonl"
    monkeypatch.setenv("HWENO_TUNING_CACHE", str(cache))
    cfg = _cfg()
    spec, st = W.quadrant_vortex_2d(96, seed=7)
    outs = []
    for mode in ("default", "timed", "cached"):
        with hw.Handle([spec], cfg) as h:
            h.set_state(0, st)
            if mode != "default":
                h.set_tuning(use_graph=0)
                t = h.autotune()
                assert t.use_graph == 0
                assert t.source == (hw.TUNED_BY_TIMING if mode == "timed" else hw.TUNED_FROM_CACHE)
                assert h.tuning().source == t.source
            for _ in range(3):
                h.step()
            outs.append(h.get_state(0)[0])
            if mode == "timed":
                timed = (t.tile_rows, t.grid_blocks, t.variant)
                # the winner is one of the listed candidates, all eager
                cands = h.tuning_candidates()
                assert timed in {(c.tile_rows, c.grid_blocks, c.variant) for c in cands}
                assert all(c.use_graph == 0 for c in cands)
            elif mode == "cached":
                assert (t.tile_rows, t.grid_blocks, t.variant) == timed
    lines = cache.read_text().splitlines()
    assert len(lines) == 1 and '"tile_rows"' in lines[0] and "|dim2|flux2|" in lines[0]
    for o in outs[1:]:
        np.testing.assert_array_equal(o, outs[0])


def test_light_step_counts_and_final_time():
    """Several problems with different end times run to their ends: every
    problem lands exactly on its t_end, and the step count equals the
    oracle's longest run (the counters the dt and finish kernels keep)."""
    cfg = _cfg()
    specs, states, ends = [], [], [0.012, 0.03, 0.021]
    for k, te in enumerate(ends):
        spec, st = W.quadrant_vortex_2d(32 + 8 * k, seed=20 + k, t_end=te)
        specs.append(spec)
        states.append(st)
    with hw.Handle(specs, cfg) as h:
        for k, st in enumerate(states):
            h.set_state(k, st)
        n = h.run_to_time()
        finals = [h.get_state(k) for k in range(len(specs))]
    counts = []
    for k, (spec, st) in enumerate(zip(specs, states)):
        ref, m = O.run(oproblem(spec, cfg), st, 0.0, spec.t_end, CFL)
        counts.append(m)
        g, t = finals[k]
        assert t == spec.t_end
        assert scaled_err(g, ref, natural_scales(spec, st)) < 1e-10
    assert n == max(counts)


@pytest.mark.parametrize("graph", [1, 0])
def test_steps_equal_single_steps(graph):
    """hweno_steps (runs of 8 steps replayed as one graph) takes the same
    steps as hweno_step called one at a time: the same bits, the same times,
    and a problem that reaches its t_end on the way stays there."""
    cfg = _cfg()
    spec0, s0 = W.quadrant_vortex_2d(64, seed=31)
    spec1, s1 = W.quadrant_vortex_2d(40, seed=32, t_end=0.01)
    finals = []
    for batched in (True, False):
        with hw.Handle([spec0, spec1], cfg) as h:
            h.set_tuning(use_graph=graph)
            h.set_state(0, s0)
            h.set_state(1, s1)
            if batched:
                h.steps(5)
                h.steps(14)
            else:
                for _ in range(19):
                    h.step()
            finals.append([h.get_state(k) for k in range(2)])
    for k in range(2):
        (a, ta), (b, tb) = finals[0][k], finals[1][k]
        assert ta == tb and np.array_equal(a, b), k
    assert finals[0][1][1] == spec1.t_end
    ref, n = O.run(oproblem(spec1, cfg), s1, 0.0, spec1.t_end, CFL)
    assert n < 19
    assert scaled_err(finals[0][1][0], ref, natural_scales(spec1, s1)) < 1e-10


def test_profiled_counters_cover_every_tuner_candidate():
    """The bench line's measured traffic comes from a table of counters
    (bench.py's PROFILED) taken for every launch configuration the tuner can
    choose; while the kernel sources are the profiled ones, every candidate
    hweno_tuning_candidates lists for the benchmark workloads must be in it,
    or the line would report no traffic for that choice."""
    import bench
    if bench.kernel_sources_hash() != bench.PROFILED_SOURCES:
        pytest.skip("kernel sources changed since the counters were taken")
    import dataclasses
    spec, _ = W.quadrant_vortex_2d(64, seed=7)
    specs2d = [dataclasses.replace(spec, nx=2048, ny=2048)]   # the benchmark's size
    missing = []
    for name, prec, charwise in (("f32acc64", hw.F32_ACC64, 0), ("f64", hw.F64, 0),
                                 ("f32acc64_characteristic", hw.F32_ACC64, 1)):
        cfg = hw.default_config(2, precision=prec, gauss_q=2, cfl=0.5, characteristic=charwise)
        with hw.Handle(specs2d, cfg) as h:
            for c in h.tuning_candidates():
                key = (name, c.tile_rows, c.grid_blocks, c.variant)
                if key not in bench.PROFILED:
                    missing.append(key)
    entries = W.batched_1d(seed=1, nprob=4096)
    with hw.Handle([e[0] for e in entries], hw.default_config(1, precision=hw.F32_ACC64)) as h:
        for c in h.tuning_candidates():
            if ("batched_1d", 0, c.grid_blocks, c.variant) not in bench.PROFILED:
                missing.append(("batched_1d", c.grid_blocks, c.variant))
    assert not missing, missing
