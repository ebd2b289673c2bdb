"""Seeded synthetic workloads and the projection of initial data onto the
unknowns of the scheme.

This module holds no arithmetic of the HWENO method itself: it only builds
initial conditions u(x, 0) = u0(x) (the problem statement of Sec. 1) as the
cell averages and derivative averages the scheme evolves, for the paper's
accuracy examples (Sec. 3.1, Examples 1-4) and for seeded synthetic
workloads of the shapes the benchmark measures.  Both the GPU tests and the
oracle tests take their inputs from here.

Unknowns (Sec. 2.1 and 2.2):
  1D  u-bar = cell mean of u,  v-bar = cell mean of u_x
      = (u(x_{i+1/2}) - u(x_{i-1/2})) / dx  (one-sided traces from inside).
  2D  u-bar = cell mean of u,
      v-bar = (1/dy) * integral of u_x over the cell
            = (1/dy) * int [u(x_{i+1/2}, y) - u(x_{i-1/2}, y)] dy,
      w-bar = (1/dx) * integral of u_y over the cell, likewise.
State arrays: float64, shape (nvar, K, ny, nx), nvar = 2 (1D) or 3 (2D).
Random draws use numpy's default_rng (PCG64), in the order documented per
workload.
"""
from __future__ import annotations

from dataclasses import dataclass, field, replace
from typing import Callable, List, Optional, Tuple

import numpy as np

ADVECTION, BURGERS, EULER = 0, 1, 2
PERIODIC, TRANSMISSIVE, REFLECTIVE = 0, 1, 2
GAS_GAMMA = 1.4


@dataclass
class Spec:
    """A problem u_t + div F(u) = 0 on a uniform rectangle (library neutral)."""
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
    gas_gamma: float = GAS_GAMMA
    adv: Tuple[float, float] = (1.0, 1.0)
    t_end: float = 0.0
    name: str = ""

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

    @property
    def ncells(self) -> int:
        return self.nx * self.ny


def _gauss(n: int):
    """Gauss-Legendre nodes and weights on [0, 1]."""
    x, w = np.polynomial.legendre.leggauss(n)
    return 0.5 * (x + 1.0), 0.5 * w


def conserved_1d(rho, u, p, gamma=GAS_GAMMA):
    return np.stack([rho, rho * u, p / (gamma - 1.0) + 0.5 * rho * u * u])


def conserved_2d(rho, u, v, p, gamma=GAS_GAMMA):
    return np.stack([rho, rho * u, rho * v, p / (gamma - 1.0) + 0.5 * rho * (u * u + v * v)])


# ---------------------------------------------------------------------------
# projection of u0 onto (u-bar, v-bar[, w-bar])
# ---------------------------------------------------------------------------

def project_1d(spec: Spec, u0: Callable, nq: int = 8) -> np.ndarray:
    """u0(x, cell_index) -> array (K, len(x)); the cell index selects the
    one-sided branch of piecewise data so traces are taken from inside."""
    nx, dx = spec.nx, spec.dx
    xl = spec.xlo + dx * np.arange(nx)
    cell = np.arange(nx)
    gx, gw = _gauss(nq)
    ubar = np.zeros((spec.K, nx))
    for xq, wq in zip(gx, gw):
        ubar += wq * np.asarray(u0(xl + xq * dx, cell), dtype=np.float64).reshape(spec.K, nx)
    right = np.asarray(u0(xl + dx, cell), dtype=np.float64).reshape(spec.K, nx)
    left = np.asarray(u0(xl, cell), dtype=np.float64).reshape(spec.K, nx)
    vbar = (right - left) / dx
    st = np.zeros(spec.shape())
    st[0, :, 0, :] = ubar
    st[1, :, 0, :] = vbar
    return st


def project_2d(spec: Spec, u0: Callable, nq: int = 4) -> np.ndarray:
    """u0(X, Y, I, J) -> array (K, *X.shape); (I, J) is the cell of each point,
    so piecewise data are evaluated on the cell's own branch (inner traces)."""
    nx, ny, dx, dy = spec.nx, spec.ny, spec.dx, spec.dy
    K = spec.K
    J, I = np.meshgrid(np.arange(ny), np.arange(nx), indexing="ij")
    XL = spec.xlo + dx * I
    YL = spec.ylo + dy * J
    g, w = _gauss(nq)
    st = np.zeros(spec.shape())
    for a in range(nq):
        for b in range(nq):
            val = np.asarray(u0(XL + g[a] * dx, YL + g[b] * dy, I, J), dtype=np.float64)
            st[0] += (w[a] * w[b]) * val.reshape(K, ny, nx)
    for b in range(nq):
        r = np.asarray(u0(XL + dx, YL + g[b] * dy, I, J), dtype=np.float64).reshape(K, ny, nx)
        l = np.asarray(u0(XL, YL + g[b] * dy, I, J), dtype=np.float64).reshape(K, ny, nx)
        st[1] += w[b] * (r - l)          # (1/dy) int [u]_x dy, scaled average
    for a in range(nq):
        t = np.asarray(u0(XL + g[a] * dx, YL + dy, I, J), dtype=np.float64).reshape(K, ny, nx)
        s = np.asarray(u0(XL + g[a] * dx, YL, I, J), dtype=np.float64).reshape(K, ny, nx)
        st[2] += w[a] * (t - s)
    return st


# ---------------------------------------------------------------------------
# the paper's smooth examples (Sec. 3.1) and the linear advection case
# ---------------------------------------------------------------------------

def advection_1d(nx: int, t_end: float = 2.0) -> Tuple[Spec, np.ndarray]:
    """u_t + u_x = 0 on periodic [0, 2], u0 = 1 + 0.5 sin(pi x); exact cell
    averages and derivative means in closed form."""
    spec = Spec(dim=1, flux=ADVECTION, nx=nx, xlo=0.0, xhi=2.0, adv=(1.0, 0.0),
                t_end=t_end, name=f"advection-1d-{nx}")
    dx = spec.dx
    xl = dx * np.arange(nx)
    xr = xl + dx
    st = np.zeros(spec.shape())
    st[0, 0, 0] = 1.0 + 0.5 * (np.cos(np.pi * xl) - np.cos(np.pi * xr)) / (np.pi * dx)
    st[1, 0, 0] = 0.5 * (np.sin(np.pi * xr) - np.sin(np.pi * xl)) / dx
    return spec, st


def burgers_1d(nx: int) -> Tuple[Spec, np.ndarray]:
    """Example 1: u_t + (u^2/2)_x = 0, periodic [0, 2], u0 = 0.5 + sin(pi x)."""
    spec = Spec(dim=1, flux=BURGERS, nx=nx, xlo=0.0, xhi=2.0, t_end=0.5 / np.pi,
                name=f"burgers-1d-{nx}")
    return spec, project_1d(spec, lambda x, c: 0.5 + np.sin(np.pi * x))


def euler_1d_smooth(nx: int) -> Tuple[Spec, np.ndarray]:
    """Example 2: rho = 1 + 0.2 sin(pi x), mu = p = 1 on periodic [0, 2]."""
    spec = Spec(dim=1, flux=EULER, nx=nx, xlo=0.0, xhi=2.0, t_end=2.0,
                name=f"euler-1d-smooth-{nx}")

    def u0(x, c):
        rho = 1.0 + 0.2 * np.sin(np.pi * x)
        return conserved_1d(rho, np.ones_like(x), np.ones_like(x))
    return spec, project_1d(spec, u0)


def burgers_2d(n: int, gauss_nq: int = 4) -> Tuple[Spec, np.ndarray]:
    """Example 3: 2D Burgers on periodic [0,4]^2, u0 = 0.5 + sin(0.5 pi (x+y))."""
    spec = Spec(dim=2, flux=BURGERS, nx=n, ny=n, xlo=0.0, xhi=4.0, ylo=0.0, yhi=4.0,
                t_end=0.5 / np.pi, name=f"burgers-2d-{n}")
    return spec, project_2d(spec, lambda X, Y, I, J: (0.5 + np.sin(0.5 * np.pi * (X + Y)))[None],
                            nq=gauss_nq)


def euler_2d_smooth(n: int) -> Tuple[Spec, np.ndarray]:
    """Example 4: rho = 1 + 0.2 sin(pi (x+y)), mu = nu = p = 1, periodic [0,2]^2."""
    spec = Spec(dim=2, flux=EULER, nx=n, ny=n, xlo=0.0, xhi=2.0, ylo=0.0, yhi=2.0,
                t_end=2.0, name=f"euler-2d-smooth-{n}")

    def u0(X, Y, I, J):
        rho = 1.0 + 0.2 * np.sin(np.pi * (X + Y))
        one = np.ones_like(X)
        return conserved_2d(rho, one, one, one)
    return spec, project_2d(spec, u0)


def advection_2d(n: int, a=(1.0, 0.5)) -> Tuple[Spec, np.ndarray]:
    """Smooth 2D linear advection on periodic [0,2]^2 (scalar test problem)."""
    spec = Spec(dim=2, flux=ADVECTION, nx=n, ny=n, xlo=0.0, xhi=2.0, ylo=0.0, yhi=2.0,
                adv=tuple(a), t_end=1.0, name=f"advection-2d-{n}")
    return spec, project_2d(spec, lambda X, Y, I, J: (1.0 + 0.5 * np.sin(np.pi * X)
                                                      * np.cos(np.pi * Y))[None])


# ---------------------------------------------------------------------------
# seeded Riemann-type workloads
# ---------------------------------------------------------------------------

def _draw_state_1d(rng):
    # order: rho in [0.1, 1], u in [-1, 1], p in [0.1, 1]
    return rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(0.1, 1.0)


def riemann_1d(seed: int, nx: int = 4000, t_end: float = 0.2) -> Tuple[Spec, np.ndarray]:
    """1D Euler Riemann problem on [0,1], transmissive, interface x = 0.5.
    Draws: (rhoL, uL, pL, rhoR, uR, pR)."""
    rng = np.random.default_rng(seed)
    L = _draw_state_1d(rng)
    R = _draw_state_1d(rng)
    spec = Spec(dim=1, flux=EULER, nx=nx, xlo=0.0, xhi=1.0, bc_x=TRANSMISSIVE,
                t_end=t_end, name=f"riemann-1d-s{seed}-{nx}")
    half = nx // 2 if nx % 2 == 0 else None

    def u0(x, c):
        if half is not None:
            left = c < half             # interface on the face between cells
        else:
            left = (spec.xlo + (c + 0.5) * spec.dx) < 0.5
        rho = np.where(left, L[0], R[0])
        u = np.where(left, L[1], R[1])
        p = np.where(left, L[2], R[2])
        return conserved_1d(rho, u, p)
    return spec, project_1d(spec, u0)


def _piecewise_average_1d(spec: Spec, cuts, states, k, phi, nq=6):
    """Exact (Gauss per smooth piece) projection of piecewise data whose
    pieces have constant (u, p) and density rho_s * (1 + 0.2 sin(2 pi k x + phi))."""
    nx, dx = spec.nx, spec.dx
    edges = np.concatenate([[spec.xlo], np.asarray(cuts, dtype=np.float64), [spec.xhi]])
    xl = spec.xlo + dx * np.arange(nx)
    xr = xl + dx
    gx, gw = _gauss(nq)

    def cons(x, s):
        rho = states[s][0] * (1.0 + 0.2 * np.sin(2.0 * np.pi * k * x + phi))
        return conserved_1d(rho, np.full_like(x, states[s][1]), np.full_like(x, states[s][2]))

    ubar = np.zeros((3, nx))
    for s in range(len(states)):
        a = np.clip(edges[s], xl, xr)
        b = np.clip(edges[s + 1], xl, xr)
        length = b - a
        m = length > 0
        if not np.any(m):
            continue
        for xq, wq in zip(gx, gw):
            xs = a[m] + xq * length[m]
            ubar[:, m] += (wq * length[m] / dx) * cons(xs, s)
    # face traces from inside each cell: piece containing the face point,
    # taken on the side of the cell
    seg_of_right = np.searchsorted(edges, xr, side="left") - 1
    seg_of_left = np.searchsorted(edges, xl, side="right") - 1
    seg_of_right = np.clip(seg_of_right, 0, len(states) - 1)
    seg_of_left = np.clip(seg_of_left, 0, len(states) - 1)
    right = np.zeros((3, nx))
    left = np.zeros((3, nx))
    for s in range(len(states)):
        mr = seg_of_right == s
        ml = seg_of_left == s
        if np.any(mr):
            right[:, mr] = cons(xr[mr], s)
        if np.any(ml):
            left[:, ml] = cons(xl[ml], s)
    st = np.zeros(spec.shape())
    st[0, :, 0, :] = ubar
    st[1, :, 0, :] = (right - left) / dx
    return st


def piecewise_1d(spec: Spec, cuts, pieces, nq: int = 8) -> np.ndarray:
    """1D Euler data made of pieces separated by the points `cuts`; piece s is
    a callable x -> (rho, u, p) (arrays).  Averages are Gauss sums over each
    piece's part of a cell (exact up to the rule's order on smooth pieces),
    and the derivative mean is the difference of the face traces taken from
    inside the cell, divided by dx."""
    nx, dx = spec.nx, spec.dx
    edges = np.concatenate([[spec.xlo], np.asarray(cuts, dtype=np.float64), [spec.xhi]])
    xl = spec.xlo + dx * np.arange(nx)
    xr = xl + dx
    gx, gw = _gauss(nq)

    def cons(x, s):
        rho, u, p = pieces[s](x)
        return conserved_1d(rho + 0 * x, u + 0 * x, p + 0 * x, spec.gas_gamma)

    ubar = np.zeros((3, nx))
    for s in range(len(pieces)):
        a = np.clip(edges[s], xl, xr)
        b = np.clip(edges[s + 1], xl, xr)
        length = b - a
        m = length > 0
        for xq, wq in zip(gx, gw):
            ubar[:, m] += (wq * length[m] / dx) * cons(a[m] + xq * length[m], s)
    seg_r = np.clip(np.searchsorted(edges, xr, side="left") - 1, 0, len(pieces) - 1)
    seg_l = np.clip(np.searchsorted(edges, xl, side="right") - 1, 0, len(pieces) - 1)
    right = np.zeros((3, nx))
    left = np.zeros((3, nx))
    for s in range(len(pieces)):
        mr, ml = seg_r == s, seg_l == s
        right[:, mr] = cons(xr[mr], s)
        left[:, ml] = cons(xl[ml], s)
    st = np.zeros(spec.shape())
    st[0, :, 0, :] = ubar
    st[1, :, 0, :] = (right - left) / dx
    return st


def lax_1d(nx: int = 100) -> Tuple[Spec, np.ndarray]:
    """Lax shock tube (Sec. 3.2): [-0.5, 0.5], jump at 0, T = 0.16; the waves
    stay inside the domain, so the inflow/outflow ends are transmissive."""
    spec = Spec(dim=1, flux=EULER, nx=nx, xlo=-0.5, xhi=0.5, bc_x=TRANSMISSIVE, t_end=0.16,
                name=f"lax-1d-{nx}")
    return spec, piecewise_1d(spec, [0.0], [lambda x: (0.445, 0.698, 3.528),
                                            lambda x: (0.5, 0.0, 0.571)])


def blast_1d(nx: int = 800) -> Tuple[Spec, np.ndarray]:
    """Interacting blast waves (Sec. 3.2): [0, 1], pressures 1000 / 0.01 /
    100 with cuts at 0.1 and 0.9, density 1 at rest, solid walls at both
    ends, T = 0.038."""
    spec = Spec(dim=1, flux=EULER, nx=nx, xlo=0.0, xhi=1.0, bc_x=REFLECTIVE, t_end=0.038,
                name=f"blast-1d-{nx}")
    return spec, piecewise_1d(spec, [0.1, 0.9], [lambda x: (1.0, 0.0, 1000.0),
                                                 lambda x: (1.0, 0.0, 0.01),
                                                 lambda x: (1.0, 0.0, 100.0)])


def shu_osher_1d(nx: int = 400) -> Tuple[Spec, np.ndarray]:
    """Shu-Osher shock/entropy-wave problem (Sec. 3.2): [-5, 5], shock at
    x = -4, density 1 + 0.2 sin(5 pi x) ahead of it, outflow ends, T = 1.8."""
    spec = Spec(dim=1, flux=EULER, nx=nx, xlo=-5.0, xhi=5.0, bc_x=TRANSMISSIVE, t_end=1.8,
                name=f"shu-osher-1d-{nx}")
    return spec, piecewise_1d(spec, [-4.0], [
        lambda x: (3.857143, 2.629369, 10.33333),
        lambda x: (1.0 + 0.2 * np.sin(5.0 * np.pi * x), 0.0, 1.0)])


def batched_1d(seed: int = 1, nprob: int = 4096, nmin: int = 256, nmax: int = 8192,
               t_end: float = 0.2):
    """Independent 1D Euler problems of uneven size on [0,1], transmissive.
    Per problem, draws in order: N ~ U{nmin..nmax}; number of jumps ~ U{1..3};
    jump positions ~ U(0.05, 0.95) (sorted); one state per piece as in the
    Riemann workload; k ~ U{1..8}; phi ~ U[0, 2 pi)."""
    rng = np.random.default_rng(seed)
    out = []
    for pidx in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        nj = int(rng.integers(1, 4))
        cuts = np.sort(rng.uniform(0.05, 0.95, size=nj))
        states = [_draw_state_1d(rng) for _ in range(nj + 1)]
        k = int(rng.integers(1, 9))
        phi = float(rng.uniform(0.0, 2.0 * np.pi))
        spec = Spec(dim=1, flux=EULER, nx=n, xlo=0.0, xhi=1.0, bc_x=TRANSMISSIVE,
                    t_end=t_end, name=f"batched-1d-s{seed}-p{pidx}")
        out.append((spec, None, (cuts, states, k, phi)))
    return out


def batched_1d_state(entry) -> np.ndarray:
    spec, _, (cuts, states, k, phi) = entry
    return _piecewise_average_1d(spec, cuts, states, k, phi)


def _draw_state_2d(rng):
    # order: rho in [0.1, 1], u in [-1, 1], v in [-1, 1], p in [0.1, 1]
    return (rng.uniform(0.1, 1.0), rng.uniform(-1.0, 1.0), rng.uniform(-1.0, 1.0),
            rng.uniform(0.1, 1.0))


def quadrant_vortex_2d(n: int = 2048, seed: int = 7, t_end: float = 0.1,
                       vortex: bool = True, nq: int = 3) -> Tuple[Spec, np.ndarray]:
    """2D Euler on periodic [0,1]^2: four constant quadrant states split at
    x = 0.5, y = 0.5 (cell faces for even n) plus an isentropic vortex of
    strength 1 and radius 0.05.  Draws in order: the states of quadrants
    (x<.5,y<.5), (x>.5,y<.5), (x<.5,y>.5), (x>.5,y>.5), each (rho, u, v, p);
    then the vortex centre (xc, yc) ~ U[0.1, 0.4]^2."""
    rng = np.random.default_rng(seed)
    Q = [_draw_state_2d(rng) for _ in range(4)]
    xc, yc = rng.uniform(0.1, 0.4), rng.uniform(0.1, 0.4)
    spec = Spec(dim=2, flux=EULER, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0,
                t_end=t_end, name=f"quadrant-vortex-2d-s{seed}-{n}")
    g = spec.gas_gamma
    eps, R = 1.0, 0.05
    Qa = np.asarray(Q)

    def u0(X, Y, I, J):
        qx = (I >= n // 2).astype(np.int64) if n % 2 == 0 else (X >= 0.5).astype(np.int64)
        qy = (J >= n // 2).astype(np.int64) if n % 2 == 0 else (Y >= 0.5).astype(np.int64)
        q = qx + 2 * qy
        rho0, u, v, p0 = Qa[q, 0], Qa[q, 1], Qa[q, 2], Qa[q, 3]
        if vortex:
            dxv = X - xc
            dyv = Y - yc
            r2 = (dxv * dxv + dyv * dyv) / (R * R)
            e = np.exp(0.5 * (1.0 - r2))
            u = u - eps / (2.0 * np.pi) * (dyv / R) * e
            v = v + eps / (2.0 * np.pi) * (dxv / R) * e
            T0 = p0 / rho0
            T = T0 - (g - 1.0) * eps * eps / (8.0 * g * np.pi * np.pi) * e * e
            rho = rho0 * (T / T0) ** (1.0 / (g - 1.0))
            p = rho * T
        else:
            rho, p = rho0, p0
        return conserved_2d(rho, u, v, p, g)
    return spec, project_2d(spec, u0, nq=nq)


def batched_2d(seed: int = 11, nprob: int = 256, nmin: int = 128, nmax: int = 1024,
               t_end: float = 0.1):
    """Independent square 2D Euler problems on [0,1]^2.  Per problem, draws in
    order: side N ~ U{nmin..nmax}; bc_x, bc_y ~ Bernoulli(1/2) (1 =
    transmissive); kind ~ Bernoulli(1/2) (0 = quadrant Riemann, 1 = smooth
    density wave); then either the four quadrant states, or (rho0, u, v, p)
    and integer wave numbers kx, ky ~ U{1..4}."""
    rng = np.random.default_rng(seed)
    out = []
    for pidx in range(nprob):
        n = int(rng.integers(nmin, nmax + 1))
        bx, by = int(rng.integers(0, 2)), int(rng.integers(0, 2))
        kind = int(rng.integers(0, 2))
        if kind == 0:
            params = ("quadrant", [_draw_state_2d(rng) for _ in range(4)])
        else:
            st = _draw_state_2d(rng)
            kx, ky = int(rng.integers(1, 5)), int(rng.integers(1, 5))
            params = ("wave", (st, kx, ky))
        spec = Spec(dim=2, flux=EULER, nx=n, ny=n, xlo=0.0, xhi=1.0, ylo=0.0, yhi=1.0,
                    bc_x=bx, bc_y=by, t_end=t_end, name=f"batched-2d-s{seed}-p{pidx}")
        out.append((spec, None, params))
    return out


def batched_2d_state(entry) -> np.ndarray:
    """Exact projection of a batched 2D problem.  Quadrant states are constant
    in every cell (the split lies on the face nearest 0.5), so the derivative
    averages vanish.  The density wave rho0 (1 + 0.2 sin(a x + b y)),
    a = 2 pi kx, b = 2 pi ky, with constant (u, v, p) makes every conserved
    variable affine in rho, and the cell and face means of the sine are
    closed forms: mean over a cell = sin(a xc + b yc) S(a dx/2) S(b dy/2) with
    S(z) = sin(z)/z."""
    spec, _, (kind, params) = entry
    n = spec.nx
    g = spec.gas_gamma
    st = np.zeros(spec.shape())
    if kind == "quadrant":
        Qa = np.asarray(params)
        J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
        q = (I >= n // 2).astype(np.int64) + 2 * (J >= n // 2).astype(np.int64)
        st[0] = conserved_2d(Qa[q, 0], Qa[q, 1], Qa[q, 2], Qa[q, 3], g)
        return st
    (rho0, u, v, p), kx, ky = params
    dx, dy = spec.dx, spec.dy
    a, b = 2.0 * np.pi * kx, 2.0 * np.pi * ky
    sx, sy = np.sinc(a * dx / 2 / np.pi), np.sinc(b * dy / 2 / np.pi)   # sin(z)/z
    xc = spec.xlo + dx * (np.arange(n) + 0.5)
    yc = spec.ylo + dy * (np.arange(n) + 0.5)
    Y, X = np.meshgrid(yc, xc, indexing="ij")
    Bv = np.array([1.0, u, v, 0.5 * (u * u + v * v)])            # dU/drho
    A = np.array([0.0, 0.0, 0.0, p / (g - 1.0)])
    rbar = rho0 * (1.0 + 0.2 * np.sin(a * X + b * Y) * sx * sy)
    st[0] = A[:, None, None] + Bv[:, None, None] * rbar[None]
    # (1/dy) int [rho(x_{i+1/2}, y) - rho(x_{i-1/2}, y)] dy, likewise in y
    dvx = 0.2 * rho0 * sy * (np.sin(a * (X + dx / 2) + b * Y) - np.sin(a * (X - dx / 2) + b * Y))
    dvy = 0.2 * rho0 * sx * (np.sin(a * X + b * (Y + dy / 2)) - np.sin(a * X + b * (Y - dy / 2)))
    st[1] = Bv[:, None, None] * dvx[None]
    st[2] = Bv[:, None, None] * dvy[None]
    return st
