"""Brute-force restatement of the scheme from its defining conditions, for
pinning the oracle on tiny grids (test-only, numpy).

Nothing here uses Appendix A: the reconstruction polynomials are obtained by
solving the conditions of Step 1 (Sec. 2.1 and 2.2) as linear systems --
exact interpolation in 1D, equality-constrained least squares (KKT system) in
2D -- and evaluated monomial by monomial; edge integrals use numpy's
Gauss-Legendre rule.
"""
from __future__ import annotations

import numpy as np

# 2D basis in the coefficient order of Appendix A
MN = [(0, 0), (1, 0), (0, 1), (2, 0), (1, 1), (0, 2), (3, 0), (2, 1), (1, 2), (0, 3),
      (4, 0), (3, 1), (2, 2), (1, 3), (0, 4)]


def integ(k, a, b):
    """integral of t^k over [a, b]"""
    return (b ** (k + 1) - a ** (k + 1)) / (k + 1)


def p0_1d(ub, dvm, dvp):
    """Quartic matching three cell averages and the scaled derivative means of
    the two neighbours (cells centred at -1, 0, 1 in units of dx)."""
    A = np.zeros((5, 5))
    b = np.zeros(5)
    for r, k in enumerate((-1, 0, 1)):
        A[r] = [integ(l, k - 0.5, k + 0.5) for l in range(5)]
        b[r] = ub[r]
    for r, (k, val) in enumerate(((-1, dvm), (1, dvp))):
        # mean of d/dxi over the cell = p(k+1/2) - p(k-1/2)
        A[3 + r] = [(k + 0.5) ** l - (k - 0.5) ** l for l in range(5)]
        b[3 + r] = val
    return np.linalg.solve(A, b)


def p0_2d(ub9, vb4, wb4, neighbours="face"):
    """Equality-constrained least squares of Step 1 (Sec. 2.2).
    ub9: averages of the 3x3 block, row-major from (-1,-1);
    vb4, wb4: scaled derivative averages of the W, E, S, N face neighbours.
    neighbours='all8' uses derivative data of all eight neighbours instead
    (then vb4/wb4 must have 8 entries, row-major without the centre)."""
    cells = [(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
    B = np.zeros((9, 15))
    d = np.zeros(9)
    for r, (a, b) in enumerate(cells):
        B[r] = [integ(m, a - 0.5, a + 0.5) * integ(n, b - 0.5, b + 0.5) for (m, n) in MN]
        d[r] = ub9[r]
    if neighbours == "face":
        nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
    else:
        nb = [c for c in cells if c != (0, 0)]
    rows, rhs = [], []
    for t, (a, b) in enumerate(nb):
        # scaled mean of d/dxi over the cell: int_y [p(a+1/2,y) - p(a-1/2,y)] dy
        rows.append([((a + 0.5) ** m - (a - 0.5) ** m) * integ(n, b - 0.5, b + 0.5)
                     if m > 0 else 0.0 for (m, n) in MN])
        rhs.append(vb4[t])
        rows.append([((b + 0.5) ** n - (b - 0.5) ** n) * integ(m, a - 0.5, a + 0.5)
                     if n > 0 else 0.0 for (m, n) in MN])
        rhs.append(wb4[t])
    A = np.array(rows)
    y = np.array(rhs)
    # KKT: minimise |A c - y|^2 subject to B c = d
    kkt = np.zeros((15 + 9, 15 + 9))
    kkt[:15, :15] = 2 * A.T @ A
    kkt[:15, 15:] = B.T
    kkt[15:, :15] = B
    sol = np.linalg.solve(kkt, np.concatenate([2 * A.T @ y, d]))
    return sol[:15]


def eval2(C, x, y):
    u = sum(C[l] * x ** m * y ** n for l, (m, n) in enumerate(MN))
    ux = sum(C[l] * m * x ** (m - 1) * y ** n for l, (m, n) in enumerate(MN) if m > 0)
    uy = sum(C[l] * n * x ** m * y ** (n - 1) for l, (m, n) in enumerate(MN) if n > 0)
    return u, ux, uy


def fact(k):
    return float(np.prod(np.arange(1, k + 1))) if k > 1 else 1.0


def weights(beta, gam, eps, squared):
    M = len(beta) - 1
    tau = sum(abs(beta[0] - beta[m]) for m in range(1, M + 1)) / M
    den = [(b * b if squared else b) + eps for b in beta]
    wt = [gam[m] * (1 + tau * tau / den[m]) for m in range(M + 1)]
    s = sum(wt)
    return [w / s for w in wt]


def rhs_1d_scalar(ub, vb, dx, flux, dflux, alpha, gam, eps, squared=False):
    """L^u, L^v and v-hat of a periodic scalar 1D problem (every cell)."""
    n = len(ub)
    polys, vh = [], []
    for i in range(n):
        um, u0, up = ub[i - 1], ub[i], ub[(i + 1) % n]
        c0 = p0_1d([um, u0, up], dx * vb[i - 1], dx * vb[(i + 1) % n])
        c1 = np.array([u0, u0 - um, 0, 0, 0])
        c2 = np.array([u0, up - u0, 0, 0, 0])
        beta = [sum((fact(l) * c0[l]) ** 2 for l in range(1, 5)), c1[1] ** 2, c2[1] ** 2]
        w = weights(beta, gam, eps, squared)
        C = w[0] * (c0 / gam[0] - gam[1] / gam[0] * c1 - gam[2] / gam[0] * c2) \
            + w[1] * c1 + w[2] * c2
        polys.append(C)
        pv = np.polynomial.polynomial.polyval
        vh.append((pv(0.5, C) - pv(-0.5, C)) / dx)
    pv = np.polynomial.polynomial.polyval
    der = lambda C: np.polynomial.polynomial.polyder(C)
    fh, hh = np.zeros(n), np.zeros(n)
    for i in range(n):  # interface i+1/2
        CL, CR = polys[i], polys[(i + 1) % n]
        uL, uR = pv(0.5, CL), pv(-0.5, CR)
        vL, vR = pv(0.5, der(CL)) / dx, pv(-0.5, der(CR)) / dx
        fh[i] = 0.5 * (flux(uL) + flux(uR)) - 0.5 * alpha * (uR - uL)
        hh[i] = 0.5 * (dflux(uL) * vL + dflux(uR) * vR) - 0.5 * alpha * (vR - vL)
    Lu = -(fh - np.roll(fh, 1)) / dx
    Lv = -(hh - np.roll(hh, 1)) / dx
    return Lu, Lv, np.array(vh)


def rhs_2d_scalar(ub, vb, wb, dx, dy, flux, dflux, ax, ay, gam, eps, squared, Q):
    """L^u, L^v, L^w, v-hat, w-hat of a periodic scalar 2D problem; ub etc.
    have shape (ny, nx); f = g = flux (same flux in both directions)."""
    ny, nx = ub.shape
    g, gw = np.polynomial.legendre.leggauss(Q)
    g, gw = 0.5 * g, 0.5 * gw
    P = np.zeros((ny, nx, 15))
    vh = np.zeros((ny, nx))
    wh = np.zeros((ny, nx))
    K2 = [fact(m) * fact(n) for (m, n) in MN]
    for j in range(ny):
        for i in range(nx):
            U = lambda a, b: ub[(j + b) % ny, (i + a) % nx]
            V = lambda a, b: vb[(j + b) % ny, (i + a) % nx]
            Wf = lambda a, b: wb[(j + b) % ny, (i + a) % nx]
            u9 = [U(a, b) for b in (-1, 0, 1) for a in (-1, 0, 1)]
            nb = [(-1, 0), (1, 0), (0, -1), (0, 1)]
            c0 = p0_2d(u9, [V(a, b) for a, b in nb], [Wf(a, b) for a, b in nb])
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
            P[j, i] = C
            # cell integrals of the partial derivatives (scaled units)
            vh[j, i] = sum(C[l] * m * integ(m - 1, -.5, .5) * integ(n, -.5, .5)
                           for l, (m, n) in enumerate(MN) if m > 0)
            wh[j, i] = sum(C[l] * n * integ(m, -.5, .5) * integ(n - 1, -.5, .5)
                           for l, (m, n) in enumerate(MN) if n > 0)
    FX = np.zeros((3, ny, nx))   # at x_{i+1/2}
    FY = np.zeros((3, ny, nx))   # at y_{j+1/2}
    for j in range(ny):
        for i in range(nx):
            for mu in range(Q):
                uL, vxL, vyL = eval2(P[j, i], 0.5, g[mu])
                uR, vxR, vyR = eval2(P[j, (i + 1) % nx], -0.5, g[mu])
                VL, VR = vxL / dx, vxR / dx
                WL, WR = vyL / dy, vyR / dy
                FX[0, j, i] += gw[mu] * dy * (0.5 * (flux(uL) + flux(uR)) - 0.5 * ax * (uR - uL))
                FX[1, j, i] += gw[mu] * dy * (0.5 * (dflux(uL) * VL + dflux(uR) * VR) - 0.5 * ax * (VR - VL))
                FX[2, j, i] += gw[mu] * dy * (0.5 * (dflux(uL) * WL + dflux(uR) * WR) - 0.5 * ax * (WR - WL))
                uB, vxB, vyB = eval2(P[j, i], g[mu], 0.5)
                uT, vxT, vyT = eval2(P[(j + 1) % ny, i], g[mu], -0.5)
                VB, VT = vxB / dx, vxT / dx
                WB, WT = vyB / dy, vyT / dy
                FY[0, j, i] += gw[mu] * dx * (0.5 * (flux(uB) + flux(uT)) - 0.5 * ay * (uT - uB))
                FY[1, j, i] += gw[mu] * dx * (0.5 * (dflux(uB) * VB + dflux(uT) * VT) - 0.5 * ay * (VT - VB))
                FY[2, j, i] += gw[mu] * dx * (0.5 * (dflux(uB) * WB + dflux(uT) * WT) - 0.5 * ay * (WT - WB))
    dFX = FX - np.roll(FX, 1, axis=2)
    dFY = FY - np.roll(FY, 1, axis=1)
    Lu = -(dFX[0] + dFY[0]) / (dx * dy)
    Lv = -(dFX[1] + dFY[1]) / dy
    Lw = -(dFX[2] + dFY[2]) / dx
    return Lu, Lv, Lw, vh, wh
