"""Python face of the plain FP64 CPU oracle (``oracle/hweno_oracle.c``).

TEST INFRASTRUCTURE ONLY.  The oracle is the slow, obviously correct statement
of the derivative-based FV-HWENO scheme (Chen & Zhao, Sec. 2 and Appendix A)
that the GPU library is checked against.  Only the tests, the smoke check and
the CPU-baseline leg of the benchmark import this module; the GPU library and
its binding never do.

State arrays are numpy float64 of shape (nvar, K, ny, nx): nvar = 2 in 1D
(u-bar, v-bar) and 3 in 2D (u-bar, v-bar, w-bar); ny = 1 in 1D.
"""
from __future__ import annotations

import ctypes as C
import os
import subprocess
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhweno_oracle.so")
SRC_PATH = os.path.join(HERE, "hweno_oracle.c")

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2
W_PAPER, W_BETA, W_BETA2, W_LINEAR = 0, 1, 2, 3
BETA_MOMENT, BETA_CLASSICAL = 0, 1


def build(force: bool = True) -> str:
    """Compile the oracle with gcc (FP64, no FMA contraction, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        cmd = ["gcc", "-O2", "-std=c99", "-ffp-contract=off", "-fno-fast-math",
               "-fopenmp", "-shared", "-fPIC", "-Wall", "-Wno-unknown-pragmas",
               "-o", LIB_PATH + ".tmp", SRC_PATH, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(LIB_PATH + ".tmp", LIB_PATH)
    return LIB_PATH


class _Problem(C.Structure):
    _fields_ = [("dim", C.c_int), ("flux", C.c_int), ("nx", C.c_int), ("ny", C.c_int),
                ("xlo", C.c_double), ("xhi", C.c_double), ("ylo", C.c_double),
                ("yhi", C.c_double), ("bc_x", C.c_int), ("bc_y", C.c_int),
                ("gas_gamma", C.c_double), ("adv", C.c_double * 2),
                ("gauss_q", C.c_int), ("weights", C.c_int),
                ("gamma_lin", C.c_double * 5), ("eps", C.c_double), ("charwise", C.c_int),
                ("smoothness", C.c_int), ("alpha_stage", C.c_int)]


@dataclass
class Problem:
    dim: int
    flux: int
    nx: int
    ny: int = 1
    xlo: float = 0.0
    xhi: float = 1.0
    ylo: float = 0.0
    yhi: float = 1.0
    bc_x: int = PERIODIC
    bc_y: int = PERIODIC
    gas_gamma: float = 1.4
    adv: tuple = (1.0, 1.0)
    gauss_q: int = 3
    weights: int = W_PAPER
    gamma_lin: tuple = field(default=None)
    eps: float = 1e-8
    charwise: int = 0
    smoothness: int = BETA_MOMENT
    alpha_stage: int = 0

    def __post_init__(self):
        if self.gamma_lin is None:
            # Sec. 3: 1/400 on every linear polynomial, the rest on p0
            m = 2 if self.dim == 1 else 4
            self.gamma_lin = tuple([1.0 - m / 400.0] + [1.0 / 400.0] * m)

    @property
    def K(self) -> int:
        if self.flux != EULER:
            return 1
        return 3 if self.dim == 1 else 4

    @property
    def nvar(self) -> int:
        return 2 if self.dim == 1 else 3

    @property
    def dx(self) -> float:
        return (self.xhi - self.xlo) / self.nx

    @property
    def dy(self) -> float:
        return (self.yhi - self.ylo) / self.ny

    def shape(self):
        return (self.nvar, self.K, self.ny, self.nx)

    def _c(self) -> _Problem:
        g = list(self.gamma_lin) + [0.0] * (5 - len(self.gamma_lin))
        return _Problem(self.dim, self.flux, self.nx, self.ny, self.xlo, self.xhi,
                        self.ylo, self.yhi, self.bc_x, self.bc_y, self.gas_gamma,
                        (C.c_double * 2)(*self.adv), self.gauss_q, self.weights,
                        (C.c_double * 5)(*g), self.eps, int(self.charwise),
                        int(self.smoothness), int(self.alpha_stage))


_lib = None
_D = C.POINTER(C.c_double)


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build(force=False)
        L = C.CDLL(LIB_PATH)
        P = C.POINTER(_Problem)
        L.orc_recon_1d.argtypes = [P, _D, _D, C.c_double, _D]
        L.orc_recon_2d.argtypes = [P, _D, _D]
        L.orc_euler_eigen.argtypes = [P, C.c_int, _D, _D, _D, _D]
        L.orc_recon_char_1d.argtypes = [P, _D, _D, C.c_double, _D]
        L.orc_recon_char_2d.argtypes = [P, _D, C.c_int, _D]
        L.orc_smoothness_classical_1d.argtypes = [_D]
        L.orc_smoothness_classical_1d.restype = C.c_double
        L.orc_smoothness_classical_2d.argtypes = [_D]
        L.orc_smoothness_classical_2d.restype = C.c_double
        L.orc_poly2d_eval.argtypes = [_D, C.c_double, C.c_double, _D]
        L.orc_poly2d_eval.restype = None
        L.orc_flux.argtypes = [P, C.c_int, _D, _D, _D, _D]
        L.orc_alpha.argtypes = [P, _D, _D, _D, C.POINTER(C.c_longlong)]
        L.orc_dt.argtypes = [P, C.c_double, C.c_double, C.c_double, C.c_double]
        L.orc_dt.restype = C.c_double
        L.orc_rhs.argtypes = [P, _D, C.c_double, C.c_double, _D, _D]
        L.orc_step.argtypes = [P, _D, C.c_double, C.c_double, C.c_double]
        L.orc_run.argtypes = [P, _D, C.c_double, C.c_double, C.c_double, C.c_double,
                              C.POINTER(C.c_longlong)]
        L.orc_step_window.argtypes = [P, _D, C.c_double, C.c_double, C.c_double,
                                      C.c_int, C.c_int, C.c_int, C.c_int, _D]
        L.orc_rhs_window.argtypes = [P, _D, C.c_double, C.c_double, C.c_int, C.c_int,
                                     C.c_int, C.c_int, _D, _D]
        L.orc_set_threads.argtypes = [C.c_int]
        L.orc_set_threads.restype = None
        L.orc_get_threads.restype = C.c_int
        _lib = L
    return _lib


def _ptr(a: np.ndarray):
    return a.ctypes.data_as(_D)


def _f64(a) -> np.ndarray:
    return np.ascontiguousarray(a, dtype=np.float64)


class OracleError(RuntimeError):
    pass


def _check(rc: int, what: str):
    if rc != 0:
        raise OracleError(f"{what} failed with status {rc}")


def set_threads(n: int) -> None:
    lib().orc_set_threads(int(n))


def get_threads() -> int:
    return int(lib().orc_get_threads())


def recon_1d(p: Problem, ub, vb, dx: float) -> dict:
    ub, vb = _f64(ub), _f64(vb)
    out = np.zeros(25)
    pc = p._c()
    _check(lib().orc_recon_1d(C.byref(pc), _ptr(ub), _ptr(vb), dx, _ptr(out)), "recon_1d")
    return {"c0": out[0:5], "c1": out[5:7], "c2": out[7:9], "beta": out[9:12],
            "omega": out[12:15], "C": out[15:20], "u_right": out[20], "u_left": out[21],
            "ux_right": out[22], "ux_left": out[23], "vhat": out[24]}


def recon_2d(p: Problem, q) -> dict:
    q = _f64(q)
    assert q.size == 17
    out = np.zeros(54)
    pc = p._c()
    _check(lib().orc_recon_2d(C.byref(pc), _ptr(q), _ptr(out)), "recon_2d")
    return {"c0": out[0:15], "lin": out[15:27].reshape(4, 3), "beta": out[27:32],
            "omega": out[32:37], "C": out[37:52], "vhat": out[52], "what": out[53]}


def euler_eigen(p: Problem, direction: int, U):
    """(R, L, lam): right eigenvectors as the columns of R, L = R^-1, eigenvalues."""
    U = _f64(U)
    R = np.zeros((p.K, p.K))
    L = np.zeros((p.K, p.K))
    lam = np.zeros(p.K)
    pc = p._c()
    _check(lib().orc_euler_eigen(C.byref(pc), direction, _ptr(U), _ptr(R), _ptr(L), _ptr(lam)),
           "euler_eigen")
    return R, L, lam


def recon_char_1d(p: Problem, ub, vb, dx: float) -> dict:
    """ub (3, K): cells i-1, i, i+1; vb (2, K): derivative means of i-1, i+1."""
    ub, vb = _f64(ub), _f64(vb)
    assert ub.shape == (3, p.K) and vb.shape == (2, p.K)
    out = np.zeros(6 * p.K)
    pc = p._c()
    _check(lib().orc_recon_char_1d(C.byref(pc), _ptr(ub), _ptr(vb), dx, _ptr(out)),
           "recon_char_1d")
    return {"C": out[:5 * p.K].reshape(p.K, 5), "vhat": out[5 * p.K:]}


def recon_char_2d(p: Problem, q, direction: int) -> dict:
    """q (17, K): the stencil of recon_2d, one K-vector per entry."""
    q = _f64(q)
    assert q.shape == (17, p.K)
    out = np.zeros(17 * p.K)
    pc = p._c()
    _check(lib().orc_recon_char_2d(C.byref(pc), _ptr(q), direction, _ptr(out)),
           "recon_char_2d")
    K = p.K
    return {"C": out[:15 * K].reshape(K, 15), "vhat": out[15 * K:16 * K], "what": out[16 * K:]}


def smoothness_classical(c) -> float:
    """classical indicator of a polynomial: 5 (1D) or 15 (2D) coefficients"""
    c = _f64(c)
    if c.size == 5:
        return float(lib().orc_smoothness_classical_1d(_ptr(c)))
    assert c.size == 15
    return float(lib().orc_smoothness_classical_2d(_ptr(c)))


def poly2d_eval(Cc, xi: float, eta: float) -> np.ndarray:
    Cc = _f64(Cc)
    out = np.zeros(3)
    lib().orc_poly2d_eval(_ptr(Cc), xi, eta, _ptr(out))
    return out


def flux(p: Problem, direction: int, U, V=None):
    U = _f64(U)
    V = _f64(np.zeros_like(U) if V is None else V)
    f = np.zeros(p.K)
    jv = np.zeros(p.K)
    pc = p._c()
    _check(lib().orc_flux(C.byref(pc), direction, _ptr(U), _ptr(V), _ptr(f), _ptr(jv)), "flux")
    return f, jv


def alpha(p: Problem, state):
    st = _f64(state)
    ax, ay, bad = C.c_double(), C.c_double(), C.c_longlong(-1)
    pc = p._c()
    rc = lib().orc_alpha(C.byref(pc), _ptr(st), C.byref(ax), C.byref(ay), C.byref(bad))
    if rc != 0:
        raise OracleError(f"non-admissible state at cell {bad.value}")
    return ax.value, ay.value


def dt(p: Problem, ax: float, ay: float, cfl: float, exponent: float = 1.0) -> float:
    pc = p._c()
    return float(lib().orc_dt(C.byref(pc), ax, ay, cfl, exponent))


def rhs(p: Problem, state, ax: float, ay: float = 0.0):
    st = _f64(state)
    L = np.zeros_like(st)
    Uh = np.zeros_like(st)
    pc = p._c()
    _check(lib().orc_rhs(C.byref(pc), _ptr(st), ax, ay, _ptr(L), _ptr(Uh)), "rhs")
    return L, Uh


def step(p: Problem, state, ax: float, ay: float, dtv: float) -> np.ndarray:
    st = _f64(state).copy()
    pc = p._c()
    _check(lib().orc_step(C.byref(pc), _ptr(st), ax, ay, dtv), "step")
    return st


def run(p: Problem, state, t0: float, t_end: float, cfl: float, exponent: float = 1.0):
    st = _f64(state).copy()
    n = C.c_longlong(0)
    pc = p._c()
    _check(lib().orc_run(C.byref(pc), _ptr(st), t0, t_end, cfl, exponent, C.byref(n)), "run")
    return st, int(n.value)


def step_window(p: Problem, state, ax, ay, dtv, i0, j0, wi, wj) -> np.ndarray:
    st = _f64(state)
    wj_ = wj if p.dim == 2 else 1
    out = np.zeros((p.nvar, p.K, wj_, wi))
    pc = p._c()
    _check(lib().orc_step_window(C.byref(pc), _ptr(st), ax, ay, dtv, i0, j0, wi, wj_,
                                 _ptr(out)), "step_window")
    return out


def rhs_window(p: Problem, state, ax, ay, i0, j0, wi, wj):
    st = _f64(state)
    wj_ = wj if p.dim == 2 else 1
    L = np.zeros((p.nvar, p.K, wj_, wi))
    Uh = np.zeros_like(L)
    pc = p._c()
    _check(lib().orc_rhs_window(C.byref(pc), _ptr(st), ax, ay, i0, j0, wi, wj_, _ptr(L),
                                _ptr(Uh)), "rhs_window")
    return L, Uh
