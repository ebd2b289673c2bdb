"""The allocation-free step (hweno_step_noalloc) against the handle's step
(hweno_step) through the C ABI: same kernels, so the same bits, on two
calls in a row whose second problem is smaller (the fixed scratch keeps the
first call's contents), for 1D and 2D Euler in every precision, plus the
clip onto t_end, the caller's step, a finished problem and a
non-admissible input.  The size limit is checked without a GPU."""
import ctypes as C

import numpy as np
import pytest

from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W


def _handle_step(spec, cfg, st, dt=None):
    with hw.Handle([spec], cfg) as h:
        h.set_state(0, st)
        d = h.step(dt=None if dt is None else [dt], want_dt=True)[0]
        out, t = h.get_state(0)
    return out, d, t


class _Hip:
    """The HIP runtime the library is linked against (the test allocates and
    copies device memory itself; the entry point under test allocates
    nothing)."""

    def __init__(self):
        hw.lib()                        # the library's runtime is the one loaded
        self.h = C.CDLL("libamdhip64.so.7")
        self.h.hipMalloc.argtypes = [C.POINTER(C.c_void_p), C.c_size_t]
        self.h.hipFree.argtypes = [C.c_void_p]
        self.h.hipMemcpy.argtypes = [C.c_void_p, C.c_void_p, C.c_size_t, C.c_int]
        self.h.hipDeviceSynchronize.argtypes = []

    def _ok(self, rc):
        assert rc == 0, f"HIP error {rc}"

    def alloc(self, nbytes):
        p = C.c_void_p()
        self._ok(self.h.hipMalloc(C.byref(p), nbytes))
        return p.value

    def put(self, dst, a):
        a = np.ascontiguousarray(a)
        self._ok(self.h.hipMemcpy(dst, a.ctypes.data, a.nbytes, 1))   # host to device

    def get(self, src, a):
        self._ok(self.h.hipMemcpy(a.ctypes.data, src, a.nbytes, 2))   # device to host
        return a

    def sync(self):
        self._ok(self.h.hipDeviceSynchronize())

    def free(self, p):
        self._ok(self.h.hipFree(p))


def _noalloc_step(spec, cfg, st, t=0.0, dt=0.0, same_buffer=False):
    hip = _Hip()
    st = np.ascontiguousarray(st, dtype=np.float64)
    x = hip.alloc(st.nbytes)
    y = x if same_buffer else hip.alloc(st.nbytes)
    aux = hip.alloc(16)
    try:
        hip.put(x, st)
        if not same_buffer:
            hip.put(y, np.full_like(st, np.nan))
        hip.put(aux, np.array([-1.0, 0.0]))
        hip.put(aux + 8, np.array([-7], dtype=np.int64))
        hw.step_noalloc(spec, cfg, x, y, t=t, dt=dt, dt_out=aux, bad_out=aux + 8, stream=None)
        hip.sync()
        out = hip.get(y, np.empty_like(st))
        dt_got = float(hip.get(aux, np.empty(1))[0])
        bad = int(hip.get(aux + 8, np.empty(1, dtype=np.int64))[0])
    finally:
        hip.free(x)
        if not same_buffer:
            hip.free(y)
        hip.free(aux)
    return out, dt_got, bad


CASES = {
    "2d": (lambda: W.quadrant_vortex_2d(96, seed=7), lambda: W.quadrant_vortex_2d(40, seed=3)),
    "1d": (lambda: W.riemann_1d(2, nx=3000), lambda: W.riemann_1d(5, nx=700)),
}


@pytest.mark.gpu
@pytest.mark.parametrize("prec", [hw.F64, hw.F32_ACC64, hw.F32_KAHAN, hw.F32])
@pytest.mark.parametrize("case", list(CASES))
def test_noalloc_step_equals_handle_step_twice(case, prec):
    for make in CASES[case]:            # the second problem is smaller
        spec, st = make()
        kw = dict(gauss_q=2, cfl=0.5) if spec.dim == 2 else {}
        cfg = hw.default_config(spec.dim, precision=prec, **kw)
        want, dt_want, _ = _handle_step(spec, cfg, st)
        got, dt_got, bad = _noalloc_step(spec, cfg, st)
        print(f"{case} prec={prec} {spec.nx}x{spec.ny}: dt {dt_got:.6e}", flush=True)
        assert bad == -1
        assert dt_got == dt_want > 0.0
        np.testing.assert_array_equal(got, want)


@pytest.mark.gpu
def test_noalloc_options_clip_given_step_and_in_place():
    spec, st = W.quadrant_vortex_2d(64, seed=4)
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=0.5, alpha_stage=1)
    want, dt_want, _ = _handle_step(spec, cfg, st)
    got, dt_got, bad = _noalloc_step(spec, cfg, st, same_buffer=True)
    assert bad == -1 and dt_got == dt_want
    np.testing.assert_array_equal(got, want)
    # the caller's step
    want, dt_want, _ = _handle_step(spec, cfg, st, dt=1e-4)
    got, dt_got, _ = _noalloc_step(spec, cfg, st, dt=1e-4)
    assert dt_got == dt_want == 1e-4
    np.testing.assert_array_equal(got, want)
    # clipped onto t_end, and nothing left to do at t_end
    got, dt_got, _ = _noalloc_step(spec, cfg, st, t=spec.t_end - 1e-5)
    assert dt_got == pytest.approx(1e-5, rel=1e-9)
    got, dt_got, bad = _noalloc_step(spec, cfg, st, t=spec.t_end)
    assert dt_got == 0.0 and bad == -1
    np.testing.assert_array_equal(got, st)


@pytest.mark.gpu
def test_noalloc_reports_a_non_admissible_input():
    spec, st = W.quadrant_vortex_2d(48, seed=2)
    st = st.copy()
    st[0, 0, 5, 7] = -1.0           # negative density at j = 5, i = 7
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2, cfl=0.5)
    got, dt_got, bad = _noalloc_step(spec, cfg, st)
    assert bad == 5 * 48 + 7 and dt_got == 0.0
    np.testing.assert_array_equal(got, st)


def test_noalloc_rejects_problems_beyond_its_scratch_without_gpu():
    spec = W.Spec(dim=2, flux=W.EULER, nx=1024, ny=1024)
    cfg = hw.default_config(2, precision=hw.F64, gauss_q=2)
    p = hw.problem(spec)
    rc = hw.lib().hweno_step_noalloc(C.byref(p), C.byref(cfg), C.c_void_p(16), C.c_void_p(16),
                                     0.0, 0.0, None, None, None)
    assert rc == hw.ERR_ARG
    assert b"scratch" in hw.lib().hweno_last_error(None)
    rc = hw.lib().hweno_step_noalloc(C.byref(p), C.byref(cfg), None, None, 0.0, 0.0, None,
                                     None, None)
    assert rc == hw.ERR_ARG
