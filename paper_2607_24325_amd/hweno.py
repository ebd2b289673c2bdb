"""Thin ctypes binding of libhweno (include/hweno.h): argument marshalling only.

Every step of the scheme runs in the library's HIP kernels.  PyTorch provides
device memory (the workspace, device-side state buffers) and the HIP stream.
The library must have been built (``paper_2607_24325_amd/build.py``); there
is no fallback of any kind: a missing library raises.
"""
from __future__ import annotations

import ctypes as C
import os
from typing import Optional, Sequence

import numpy as np

PKG = os.path.dirname(os.path.abspath(__file__))
# HWENO_LIB selects another build of the same library (e.g. to compare builds)
LIB_PATH = os.environ.get("HWENO_LIB", os.path.join(PKG, "libhweno.so"))

OK, ERR_ARG, ERR_NONFINITE, ERR_HIP, ERR_STATE, ERR_OOM = 0, -1, -2, -3, -4, -5
ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2
F64, F32, F32_ACC64, F32_KAHAN = 0, 1, 2, 3
BETA_MOMENT, BETA_CLASSICAL = 0, 1
W_PAPER, W_BETA, W_BETA2, W_LINEAR = 0, 1, 2, 3


class hweno_problem(C.Structure):
    _fields_ = [("dim", C.c_int32), ("flux", C.c_int32), ("nx", C.c_int32), ("ny", C.c_int32),
                ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double),
                ("yhi", C.c_double), ("bc_x", C.c_int32), ("bc_y", C.c_int32),
                ("gas_gamma", C.c_double), ("adv", C.c_double * 2), ("t_end", C.c_double)]


class hweno_config(C.Structure):
    _fields_ = [("precision", C.c_int32), ("gauss_q", C.c_int32), ("weights", C.c_int32),
                ("gamma_lin", C.c_double * 5), ("eps", C.c_double), ("cfl", C.c_double),
                ("dt_exponent", C.c_double), ("characteristic", C.c_int32),
                ("smoothness", C.c_int32), ("alpha_stage", C.c_int32),
                ("reserved_", C.c_int32)]


class hweno_tuning(C.Structure):
    _fields_ = [("tile_rows", C.c_int32), ("grid_blocks", C.c_int32),
                ("use_graph", C.c_int32), ("variant", C.c_int32), ("source", C.c_int32),
                ("reserved", C.c_int32)]


TUNED_DEFAULT, TUNED_BY_CALLER, TUNED_BY_TIMING, TUNED_FROM_CACHE = 0, 1, 2, 3


class hweno_timing(C.Structure):
    _fields_ = [("total_ms", C.c_double), ("stage_ms", C.c_double), ("alpha_ms", C.c_double),
                ("other_ms", C.c_double), ("steps", C.c_int64), ("stage_launches", C.c_int64)]


class HwenoError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"[{code}] {msg}")
        self.code = code


_lib = None
EXPORTS = ["hweno_default_config", "hweno_workspace_bytes", "hweno_create", "hweno_set_state",
           "hweno_get_state", "hweno_rhs", "hweno_alpha", "hweno_step", "hweno_steps", "hweno_run_to_time",
           "hweno_sync", "hweno_get_tuning", "hweno_set_tuning", "hweno_autotune",
           "hweno_tuning_candidates",
           "hweno_timed_steps", "hweno_step_noalloc", "hweno_destroy", "hweno_last_error"]


def lib():
    """Load libhweno.so (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with paper_2607_24325_amd/build.py")
        L = C.CDLL(LIB_PATH)
        H = C.c_void_p
        P = C.POINTER
        L.hweno_default_config.argtypes = [C.c_int32, P(hweno_config)]
        L.hweno_default_config.restype = None
        L.hweno_workspace_bytes.argtypes = [P(hweno_problem), C.c_int32, P(hweno_config)]
        L.hweno_workspace_bytes.restype = C.c_size_t
        L.hweno_create.argtypes = [P(hweno_problem), C.c_int32, P(hweno_config), C.c_void_p,
                                   C.c_size_t, C.c_void_p, P(H)]
        L.hweno_set_state.argtypes = [H, C.c_int32, C.c_void_p, C.c_int32, C.c_double]
        L.hweno_get_state.argtypes = [H, C.c_int32, C.c_void_p, C.c_int32, P(C.c_double)]
        L.hweno_rhs.argtypes = [H, C.c_int32, C.c_void_p, C.c_void_p, C.c_int32]
        L.hweno_alpha.argtypes = [H, C.c_int32, P(C.c_double), P(C.c_double)]
        L.hweno_step.argtypes = [H, C.c_void_p, C.c_void_p]
        L.hweno_steps.argtypes = [H, C.c_int32]
        L.hweno_run_to_time.argtypes = [H, P(C.c_int64)]
        L.hweno_sync.argtypes = [H]
        L.hweno_get_tuning.argtypes = [H, P(hweno_tuning)]
        L.hweno_set_tuning.argtypes = [H, P(hweno_tuning)]
        L.hweno_autotune.argtypes = [H, P(hweno_tuning)]
        L.hweno_tuning_candidates.argtypes = [H, P(hweno_tuning), C.c_int32, P(C.c_int32)]
        L.hweno_timed_steps.argtypes = [H, C.c_int32, P(hweno_timing)]
        L.hweno_step_noalloc.argtypes = [P(hweno_problem), P(hweno_config), C.c_void_p,
                                         C.c_void_p, C.c_double, C.c_double, C.c_void_p,
                                         C.c_void_p, C.c_void_p]
        L.hweno_destroy.argtypes = [H]
        L.hweno_last_error.argtypes = [H]
        L.hweno_last_error.restype = C.c_char_p
        for f in EXPORTS:
            if f not in ("hweno_default_config", "hweno_workspace_bytes", "hweno_last_error"):
                getattr(L, f).restype = C.c_int
        _lib = L
    return _lib


def default_config(dim: int, **kw) -> hweno_config:
    cfg = hweno_config()
    lib().hweno_default_config(dim, C.byref(cfg))
    for k, v in kw.items():
        if k == "gamma_lin":
            vals = list(v) + [0.0] * (5 - len(v))
            cfg.gamma_lin = (C.c_double * 5)(*vals)
        else:
            setattr(cfg, k, v)
    return cfg


def problem(spec) -> hweno_problem:
    """hweno_problem from any object with the fields of workloads.Spec."""
    return hweno_problem(spec.dim, spec.flux, spec.nx, spec.ny, spec.xlo, spec.xhi, spec.ylo,
                         spec.yhi, spec.bc_x, spec.bc_y, spec.gas_gamma,
                         (C.c_double * 2)(*spec.adv), spec.t_end)


def _ptr(a) -> int:
    """Raw pointer of a numpy array or a torch tensor."""
    if isinstance(a, np.ndarray):
        return a.ctypes.data
    return a.data_ptr()


class Handle:
    """One libhweno handle over one or many problems."""

    def __init__(self, specs: Sequence, cfg: hweno_config, workspace=None, stream=None):
        self.specs = list(specs)
        n = len(self.specs)
        self._probs = (hweno_problem * n)(*[problem(s) for s in self.specs])
        self.cfg = cfg
        self._ws = workspace
        h = C.c_void_p()
        ws_ptr = _ptr(workspace) if workspace is not None else None
        ws_bytes = workspace.numel() * workspace.element_size() if workspace is not None else 0
        rc = lib().hweno_create(self._probs, n, C.byref(cfg), ws_ptr, ws_bytes, stream,
                                C.byref(h))
        if rc != OK:
            raise HwenoError(rc, lib().hweno_last_error(None).decode())
        self.h = h

    @staticmethod
    def workspace_bytes(specs: Sequence, cfg: hweno_config) -> int:
        n = len(specs)
        probs = (hweno_problem * n)(*[problem(s) for s in specs])
        return int(lib().hweno_workspace_bytes(probs, n, C.byref(cfg)))

    def _check(self, rc: int):
        if rc != OK:
            raise HwenoError(rc, lib().hweno_last_error(self.h).decode())

    def close(self):
        if getattr(self, "h", None):
            lib().hweno_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def state_shape(self, prob: int):
        s = self.specs[prob]
        return (s.nvar, s.K, s.ny, s.nx)

    def set_state(self, prob: int, state, t: float = 0.0):
        if isinstance(state, np.ndarray):
            st = np.ascontiguousarray(state, dtype=np.float64)
            assert st.shape == self.state_shape(prob)
            self._check(lib().hweno_set_state(self.h, prob, st.ctypes.data, 0, t))
        else:
            assert state.is_contiguous() and str(state.dtype) == "torch.float64"
            self._check(lib().hweno_set_state(self.h, prob, state.data_ptr(), 1, t))

    def get_state(self, prob: int, out=None):
        t = C.c_double()
        if out is None:
            out = np.empty(self.state_shape(prob))
        on_dev = 0 if isinstance(out, np.ndarray) else 1
        self._check(lib().hweno_get_state(self.h, prob, _ptr(out), on_dev, C.byref(t)))
        return out, t.value

    def time(self, prob: int) -> float:
        t = C.c_double()
        self._check(lib().hweno_get_state(self.h, prob, None, 0, C.byref(t)))
        return t.value

    def rhs(self, prob: int):
        L = np.empty(self.state_shape(prob))
        Uh = np.empty(self.state_shape(prob))
        self._check(lib().hweno_rhs(self.h, prob, L.ctypes.data, Uh.ctypes.data, 0))
        return L, Uh

    def alpha(self, prob: int):
        ax, ay = C.c_double(), C.c_double()
        self._check(lib().hweno_alpha(self.h, prob, C.byref(ax), C.byref(ay)))
        return ax.value, ay.value

    def step(self, dt: Optional[Sequence[float]] = None, want_dt: bool = False):
        n = len(self.specs)
        dtin = None if dt is None else np.ascontiguousarray(dt, dtype=np.float64)
        dtout = np.zeros(n) if want_dt else None
        self._check(lib().hweno_step(self.h, None if dtin is None else dtin.ctypes.data,
                                     None if dtout is None else dtout.ctypes.data))
        return dtout

    def steps(self, n: int):
        """n steps with the CFL rule (enqueued; runs of 8 as one graph)."""
        self._check(lib().hweno_steps(self.h, int(n)))

    def run_to_time(self) -> int:
        steps = C.c_int64()
        self._check(lib().hweno_run_to_time(self.h, C.byref(steps)))
        return int(steps.value)

    def sync(self):
        self._check(lib().hweno_sync(self.h))

    def tuning(self) -> hweno_tuning:
        t = hweno_tuning()
        self._check(lib().hweno_get_tuning(self.h, C.byref(t)))
        return t

    def set_tuning(self, tile_rows=None, grid_blocks=None, use_graph=None, variant=None):
        t = self.tuning()
        if tile_rows is not None:
            t.tile_rows = tile_rows
        if grid_blocks is not None:
            t.grid_blocks = grid_blocks
        if use_graph is not None:
            t.use_graph = use_graph
        if variant is not None:
            t.variant = variant
        self._check(lib().hweno_set_tuning(self.h, C.byref(t)))

    def autotune(self) -> hweno_tuning:
        t = hweno_tuning()
        self._check(lib().hweno_autotune(self.h, C.byref(t)))
        return t

    def tuning_candidates(self):
        """The launch configurations autotune() times, in its order."""
        n = C.c_int32()
        self._check(lib().hweno_tuning_candidates(self.h, None, 0, C.byref(n)))
        out = (hweno_tuning * n.value)()
        self._check(lib().hweno_tuning_candidates(self.h, out, n.value, C.byref(n)))
        return list(out)

    def tuned_from_cache(self) -> bool:
        return self.tuning().source == TUNED_FROM_CACHE

    def timed_steps(self, nsteps: int, allow_nonfinite: bool = False) -> hweno_timing:
        """Per-kernel timing of nsteps eager steps.  With allow_nonfinite, a
        problem that became non-admissible (and was frozen) does not raise:
        the timing of the steps that ran is returned."""
        t = hweno_timing()
        rc = lib().hweno_timed_steps(self.h, nsteps, C.byref(t))
        if not (allow_nonfinite and rc == ERR_NONFINITE):
            self._check(rc)
        return t

    def failed_problems(self):
        """Indices of the problems frozen because their state became
        non-admissible."""
        bad = []
        for i in range(len(self.specs)):
            t = C.c_double()
            if lib().hweno_get_state(self.h, i, None, 0, C.byref(t)) == ERR_NONFINITE:
                bad.append(i)
        return bad


def _dev_ptr(a):
    """Device address of a torch CUDA tensor, or an address given as an int."""
    if a is None or isinstance(a, int):
        return a
    assert a.is_cuda and a.is_contiguous()
    return a.data_ptr()


def step_noalloc(spec, cfg: hweno_config, state_in, state_out, t: float = 0.0,
                 dt: float = 0.0, dt_out=None, bad_out=None, stream=None) -> None:
    """hweno_step_noalloc: one step of one problem on device memory (float64
    states in the boundary layout; dt_out one float64 and bad_out one int64
    on the device, or None), given as torch CUDA tensors or raw device
    addresses.  Only enqueues on `stream`."""
    for a in (state_in, state_out):
        assert isinstance(a, int) or str(a.dtype) == "torch.float64"
    p = problem(spec)
    rc = lib().hweno_step_noalloc(C.byref(p), C.byref(cfg), _dev_ptr(state_in),
                                  _dev_ptr(state_out), float(t), float(dt), _dev_ptr(dt_out),
                                  _dev_ptr(bad_out), stream)
    if rc != OK:
        raise HwenoError(rc, lib().hweno_last_error(None).decode())
