"""Brute-force restatement of the scheme for systems and for every boundary
type but the solid wall, written independently of the oracle (test-only,
numpy).

What is independent here, and how:
  * ghost cells come from numpy's own padding (``np.pad`` with mode 'wrap'
    for periodic and 'edge' for transmissive, applied axis by axis, so that
    a 2D corner takes the cell both axis maps point to), not from an index
    map;
  * the Jacobian-vector products of the Euler flux are complex-step
    derivatives of the flux itself, J(U) V = Im F(U + i h V) / h with h tiny
    (exact to rounding for a rational function; no chain rule written out);
  * the Lax-Friedrichs speed is the spectral radius of that Jacobian, from
    ``np.linalg.eigvals``, not a sound-speed formula;
  * the reconstruction solves the conditions of Step 1 (Sec. 2.1 and 2.2) as
    linear systems (``bruteforce.p0_1d`` / ``p0_2d``) and evaluates the
    polynomials monomial by monomial; edge integrals use numpy's
    Gauss-Legendre rule.

State arrays have the oracle's shape (nvar, K, ny, nx).
"""
from __future__ import annotations

import numpy as np

from bruteforce import MN, eval2, fact, integ, p0_1d, p0_2d, weights

GAMMA = 1.4


def euler_flux(U, direction: int, gamma: float = GAMMA):
    """Physical Euler flux of the conserved state U (K = 3 in 1D, 4 in 2D),
    written through the primitive variables; valid for complex U."""
    K = len(U)
    rho, E = U[0], U[K - 1]
    vel = [U[1] / rho] + ([U[2] / rho] if K == 4 else [])
    pr = (gamma - 1.0) * (E - 0.5 * rho * sum(w * w for w in vel))
    vn = vel[direction]
    F = [rho * vn]
    for d in range(len(vel)):
        F.append(rho * vel[d] * vn + (pr if d == direction else 0.0))
    F.append((E + pr) * vn)
    return np.array(F)


def scalar_flux(kind: str, a=(1.0, 1.0)):
    if kind == "burgers":
        return lambda U, direction: np.array([0.5 * U[0] * U[0]])
    return lambda U, direction: np.array([a[direction] * U[0]])


def jvp(F, U, V, direction: int, h: float = 1e-30):
    """(dF/dU)(U) V by the complex step."""
    Uc = np.asarray(U, dtype=complex) + 1j * h * np.asarray(V, dtype=float)
    return np.imag(F(Uc, direction)) / h


def jacobian(F, U, direction: int):
    K = len(U)
    return np.column_stack([jvp(F, U, np.eye(K)[k], direction) for k in range(K)])


def spectral_radius(F, U, direction: int) -> float:
    return float(np.max(np.abs(np.linalg.eigvals(jacobian(F, U, direction)))))


def speeds(F, st):
    """Largest spectral radius of the flux Jacobians over the cell averages."""
    nvar, K, ny, nx = st.shape
    ax = ay = 0.0
    for j in range(ny):
        for i in range(nx):
            U = st[0, :, j, i]
            ax = max(ax, spectral_radius(F, U, 0))
            if nvar == 3:
                ay = max(ay, spectral_radius(F, U, 1))
    return ax, ay


MODES = {0: "wrap", 1: "edge"}   # periodic, transmissive


def pad2(a, gx, gy, bc_x, bc_y):
    """Two ghost layers on each side of a (ny, nx) plane (gy = 0 in 1D)."""
    if gy:
        a = np.pad(a, ((gy, gy), (0, 0)), mode=MODES[bc_y])
    return np.pad(a, ((0, 0), (gx, gx)), mode=MODES[bc_x])


def rhs_1d(F, st, dx, alpha, gam, eps, bc, squared=False, pad_derivative=None):
    """L = (L^u, L^v) and U-hat = (u-bar, v-hat) of a 1D problem.
    pad_derivative: an alternative ghost fill of the derivative averages
    (a (1, n) plane -> (1, n + 4)), to show what the tests can see."""
    _, K, _, n = st.shape
    padv = pad_derivative or (lambda a: pad2(a, 2, 0, bc, bc))
    ub = np.stack([pad2(st[0, c], 2, 0, bc, bc)[0] for c in range(K)])
    vb = np.stack([padv(st[1, c])[0] for c in range(K)])
    pv = np.polynomial.polynomial.polyval
    der = np.polynomial.polynomial.polyder
    polys = np.zeros((n + 2, K, 5))          # cells -1 .. n (extended index e-1)
    vhat = np.zeros((K, n))
    for e in range(1, n + 3):
        for c in range(K):
            um, u0, up = ub[c, e - 1], ub[c, e], ub[c, e + 1]
            c0 = p0_1d([um, u0, up], dx * vb[c, e - 1], dx * vb[c, e + 1])
            c1 = np.array([u0, u0 - um, 0, 0, 0])
            c2 = np.array([u0, up - u0, 0, 0, 0])
            beta = [sum((fact(l) * c0[l]) ** 2 for l in range(1, 5)), c1[1] ** 2, c2[1] ** 2]
            w = weights(beta, gam, eps, squared)
            C = w[0] * (c0 / gam[0] - gam[1] / gam[0] * c1 - gam[2] / gam[0] * c2) \
                + w[1] * c1 + w[2] * c2
            polys[e - 1, c] = C
            if 2 <= e <= n + 1:
                vhat[c, e - 2] = (pv(0.5, C) - pv(-0.5, C)) / dx
    fh = np.zeros((K, n + 1))
    hh = np.zeros((K, n + 1))
    for k in range(n + 1):                    # interface between cells k-1 and k
        CL, CR = polys[k], polys[k + 1]
        uL = np.array([pv(0.5, CL[c]) for c in range(K)])
        uR = np.array([pv(-0.5, CR[c]) for c in range(K)])
        vL = np.array([pv(0.5, der(CL[c])) for c in range(K)]) / dx
        vR = np.array([pv(-0.5, der(CR[c])) for c in range(K)]) / dx
        fh[:, k] = 0.5 * (F(uL, 0) + F(uR, 0)) - 0.5 * alpha * (uR - uL)
        hh[:, k] = 0.5 * (jvp(F, uL, vL, 0) + jvp(F, uR, vR, 0)) - 0.5 * alpha * (vR - vL)
    L = np.zeros_like(st)
    L[0, :, 0] = -(fh[:, 1:] - fh[:, :-1]) / dx
    L[1, :, 0] = -(hh[:, 1:] - hh[:, :-1]) / dx
    Uh = np.zeros_like(st)
    Uh[0] = st[0]
    Uh[1, :, 0] = vhat
    return L, Uh


def rhs_2d(F, st, dx, dy, ax, ay, gam, eps, squared, Q, bc_x, bc_y):
    """L = (L^u, L^v, L^w) and U-hat = (u-bar, v-hat, w-hat) of a 2D problem
    (eq. 2D-semi-discrete-scheme-uniform), component-wise reconstruction."""
    _, K, ny, nx = st.shape
    P = [[pad2(st[v, c], 2, 2, bc_x, bc_y) for c in range(K)] for v in range(3)]
    g, gw = np.polynomial.legendre.leggauss(Q)
    g, gw = 0.5 * g, 0.5 * gw
    K2 = [fact(m) * fact(n) for (m, n) in MN]
    nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    # polynomials of the interior cells and the ring across faces
    poly = np.zeros((ny + 2, nx + 2, K, 15))
    vh = np.zeros((K, ny, nx))
    wh = np.zeros((K, ny, nx))
    for je in range(1, ny + 3):
        for ie in range(1, nx + 3):
            for c in range(K):
                U = lambda a, b: P[0][c][je + b, ie + a]
                u9 = [U(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
                c0 = p0_2d(u9, [P[1][c][je + b, ie + a] for a, b in nb],
                           [P[2][c][je + b, ie + a] for a, b in nb])
                uc = U(0, 0)
                lin = [(uc, uc - U(-1, 0), uc - U(0, -1)), (uc, U(1, 0) - uc, uc - U(0, -1)),
                       (uc, U(1, 0) - uc, U(0, 1) - uc), (uc, uc - U(-1, 0), U(0, 1) - uc)]
                beta = [sum((K2[l] * c0[l]) ** 2 for l in range(1, 15))]
                beta += [l_[1] ** 2 + l_[2] ** 2 for l_ in lin]
                w = weights(beta, gam, eps, squared)
                C = w[0] * c0 / gam[0]
                for m in range(4):
                    cm = np.zeros(15)
                    cm[:3] = lin[m]
                    C = C - w[0] * gam[m + 1] / gam[0] * cm + w[m + 1] * cm
                poly[je - 1, ie - 1, c] = C
                if 2 <= je <= ny + 1 and 2 <= ie <= nx + 1:
                    vh[c, je - 2, ie - 2] = sum(
                        C[l] * m * integ(m - 1, -.5, .5) * integ(n, -.5, .5)
                        for l, (m, n) in enumerate(MN) if m > 0)
                    wh[c, je - 2, ie - 2] = sum(
                        C[l] * n * integ(m, -.5, .5) * integ(n - 1, -.5, .5)
                        for l, (m, n) in enumerate(MN) if n > 0)

    def edge(PL, PR, xL, yL, xR, yR, direction, alpha, length):
        """quadrature of the three Lax-Friedrichs fluxes along one edge"""
        out = np.zeros((3, K))
        for mu in range(Q):
            vl = [eval2(PL[c], *(xL(g[mu]), yL(g[mu]))) for c in range(K)]
            vr = [eval2(PR[c], *(xR(g[mu]), yR(g[mu]))) for c in range(K)]
            uL = np.array([t[0] for t in vl]); uR = np.array([t[0] for t in vr])
            VL = np.array([t[1] for t in vl]) / dx; VR = np.array([t[1] for t in vr]) / dx
            WL = np.array([t[2] for t in vl]) / dy; WR = np.array([t[2] for t in vr]) / dy
            out[0] += gw[mu] * length * (0.5 * (F(uL, direction) + F(uR, direction))
                                         - 0.5 * alpha * (uR - uL))
            out[1] += gw[mu] * length * (0.5 * (jvp(F, uL, VL, direction) + jvp(F, uR, VR, direction))
                                         - 0.5 * alpha * (VR - VL))
            out[2] += gw[mu] * length * (0.5 * (jvp(F, uL, WL, direction) + jvp(F, uR, WR, direction))
                                         - 0.5 * alpha * (WR - WL))
        return out

    half = lambda _: 0.5
    mhalf = lambda _: -0.5
    node = lambda t: t
    FX = np.zeros((3, K, ny, nx + 1))   # x-edge left of interior column i (i = 0..nx)
    FY = np.zeros((3, K, ny + 1, nx))
    for j in range(ny):
        for i in range(nx + 1):
            FX[:, :, j, i] = edge(poly[j + 1, i], poly[j + 1, i + 1], half, node, mhalf, node,
                                  0, ax, dy)
    for j in range(ny + 1):
        for i in range(nx):
            FY[:, :, j, i] = edge(poly[j, i + 1], poly[j + 1, i + 1], node, half, node, mhalf,
                                  1, ay, dx)
    dFX = FX[..., 1:] - FX[..., :-1]
    dFY = FY[:, :, 1:, :] - FY[:, :, :-1, :]
    L = np.zeros_like(st)
    L[0] = -(dFX[0] + dFY[0]) / (dx * dy)
    L[1] = -(dFX[1] + dFY[1]) / dy
    L[2] = -(dFX[2] + dFY[2]) / dx
    Uh = np.stack([st[0], vh, wh])
    return L, Uh


def ssprk3(rhs, st, dt, alphas_of):
    """One SSP-RK3 step with the modified derivatives (Sec. 2.1 / 2.2 Step 4):
    rhs(state, speeds) -> (L, U-hat); alphas_of(stage, state) gives the
    speeds of each stage."""
    L0, H0 = rhs(st, alphas_of(0, st))
    u1 = H0 + dt * L0
    L1, H1 = rhs(u1, alphas_of(1, u1))
    u2 = 0.75 * H0 + 0.25 * (H1 + dt * L1)
    L2, H2 = rhs(u2, alphas_of(2, u2))
    return H0 / 3.0 + 2.0 / 3.0 * (H2 + dt * L2)
