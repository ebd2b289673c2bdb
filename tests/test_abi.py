"""CPU checks of the C ABI: the library loads, exports every entry point the
header declares, and validates arguments before touching a GPU."""
import ctypes as C
import os
import re

import pytest

from paper_2607_24325_amd import hweno as hw
from paper_2607_24325_amd import workloads as W

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared():
    src = open(os.path.join(ROOT, "include", "hweno.h")).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(hweno_[a-z_]+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    names = declared()
    assert "hweno_create" in names and "hweno_run_to_time" in names
    L = hw.lib()
    for n in names:
        assert hasattr(L, n), n
    assert set(names) == set(hw.EXPORTS)


def test_default_config_is_the_papers():
    c1 = hw.default_config(1)
    assert list(c1.gamma_lin)[:3] == [0.995, 0.0025, 0.0025]
    c2 = hw.default_config(2)
    assert list(c2.gamma_lin) == [0.99, 0.0025, 0.0025, 0.0025, 0.0025]
    assert c2.eps == 1e-8 and c2.cfl == 0.6 and c2.gauss_q == 3 and c2.weights == hw.W_BETA


def _create(spec, cfg):
    p = hw.problem(spec)
    h = C.c_void_p()
    return hw.lib().hweno_create(C.byref(p), 1, C.byref(cfg), None, 0, None, C.byref(h))


@pytest.mark.parametrize("bad", [
    dict(gamma_lin=(0.5, 0.25, 0.2)),          # sum != 1
    dict(gamma_lin=(1.01, -0.005, -0.005)),    # negative weight
    dict(eps=0.0),
    dict(cfl=-1.0),
    dict(precision=7),
])
def test_invalid_config_rejected_without_gpu(bad):
    spec, _ = W.advection_1d(64)
    cfg = hw.default_config(1, **bad)
    assert _create(spec, cfg) == hw.ERR_ARG
    assert hw.lib().hweno_workspace_bytes(C.byref(hw.problem(spec)), 1, C.byref(cfg)) == 0
    assert len(hw.lib().hweno_last_error(None)) > 0


def test_invalid_problem_rejected_without_gpu():
    spec, _ = W.advection_1d(3)   # fewer than 4 cells
    assert _create(spec, hw.default_config(1)) == hw.ERR_ARG
    assert b"nx" in hw.lib().hweno_last_error(None)
    spec2, _ = W.burgers_2d(8)
    assert _create(spec2, hw.default_config(2, gauss_q=4)) == hw.ERR_ARG


def test_workspace_size_accounts_for_every_buffer():
    spec, _ = W.quadrant_vortex_2d(8)
    spec = W.Spec(dim=2, flux=W.EULER, nx=2048, ny=2048)
    cfg64 = hw.default_config(2, precision=hw.F64, gauss_q=2)
    cfg32 = hw.default_config(2, precision=hw.F32_ACC64, gauss_q=2)
    n = 2048 * 2048
    b64 = hw.Handle.workspace_bytes([spec], cfg64)
    b32 = hw.Handle.workspace_bytes([spec], cfg32)
    # 3 state sets of 12 values + 8 saved hats per cell, plus 2 staging copies
    assert b64 >= n * 8 * (3 * 12 + 8 + 2 * 12)
    assert b32 >= n * (3 * (4 * 8 + 8 * 4) + 8 * 4 + 2 * 12 * 8)
    assert b32 < b64
