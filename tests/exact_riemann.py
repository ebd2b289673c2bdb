"""Exact solution of the Riemann problem of the 1D Euler equations for an
ideal gas (the classical two-wave construction: a pressure function on each
side, Newton iteration for the star pressure, then sampling of the similarity
solution along x/t; Toro, Riemann Solvers and Numerical Methods for Fluid
Dynamics, ch. 4).  Test infrastructure: an independent check of the oracle
on shock-tube problems such as the Lax problem of Sec. 3.2."""
from __future__ import annotations

import math

import numpy as np


class RiemannExact:
    def __init__(self, left, right, gamma=1.4):
        self.g = gamma
        self.rl, self.ul, self.pl = left
        self.rr, self.ur, self.pr = right
        self.cl = math.sqrt(gamma * self.pl / self.rl)
        self.cr = math.sqrt(gamma * self.pr / self.rr)
        self.ps, self.us = self._star()

    def _side(self, p, r, pk, ck):
        """f_K(p) and its derivative: rarefaction for p <= p_K, shock above"""
        g = self.g
        if p <= pk:
            q = (p / pk) ** ((g - 1) / (2 * g))
            f = 2 * ck / (g - 1) * (q - 1)
            df = (1.0 / (r * ck)) * (p / pk) ** (-(g + 1) / (2 * g))
            return f, df
        A = 2.0 / ((g + 1) * r)
        B = (g - 1) / (g + 1) * pk
        s = math.sqrt(A / (p + B))
        return (p - pk) * s, s * (1 - 0.5 * (p - pk) / (p + B))

    def _star(self):
        du = self.ur - self.ul
        if 2 * (self.cl + self.cr) / (self.g - 1) <= du:
            raise ValueError("vacuum is generated")
        p = max(1e-12, 0.5 * (self.pl + self.pr))
        for _ in range(100):
            fl, dl = self._side(p, self.rl, self.pl, self.cl)
            fr, dr = self._side(p, self.rr, self.pr, self.cr)
            pn = p - (fl + fr + du) / (dl + dr)
            pn = max(pn, 1e-14)
            if abs(pn - p) <= 1e-15 * (pn + p):
                p = pn
                break
            p = pn
        fl, _ = self._side(p, self.rl, self.pl, self.cl)
        fr, _ = self._side(p, self.rr, self.pr, self.cr)
        return p, 0.5 * (self.ul + self.ur) + 0.5 * (fr - fl)

    def sample(self, s):
        """(rho, u, p) at similarity coordinate s = x / t"""
        g, ps, us = self.g, self.ps, self.us
        gm = (g - 1) / (g + 1)
        if s <= us:   # left of the contact
            r, u, p, c = self.rl, self.ul, self.pl, self.cl
            if ps > p:   # left shock
                sl = u - c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
                if s <= sl:
                    return r, u, p
                return r * (ps / p + gm) / (gm * ps / p + 1), us, ps
            shl = u - c
            cs = c * (ps / p) ** ((g - 1) / (2 * g))
            stl = us - cs
            if s <= shl:
                return r, u, p
            if s >= stl:
                return r * (ps / p) ** (1 / g), us, ps
            uu = 2 / (g + 1) * (c + (g - 1) / 2 * u + s)
            cc = 2 / (g + 1) * (c + (g - 1) / 2 * (u - s))
            return r * (cc / c) ** (2 / (g - 1)), uu, p * (cc / c) ** (2 * g / (g - 1))
        r, u, p, c = self.rr, self.ur, self.pr, self.cr
        if ps > p:   # right shock
            sr = u + c * math.sqrt((g + 1) / (2 * g) * ps / p + (g - 1) / (2 * g))
            if s >= sr:
                return r, u, p
            return r * (ps / p + gm) / (gm * ps / p + 1), us, ps
        shr = u + c
        cs = c * (ps / p) ** ((g - 1) / (2 * g))
        str_ = us + cs
        if s >= shr:
            return r, u, p
        if s <= str_:
            return r * (ps / p) ** (1 / g), us, ps
        uu = 2 / (g + 1) * (-c + (g - 1) / 2 * u + s)
        cc = 2 / (g + 1) * (c - (g - 1) / 2 * (u - s))
        return r * (cc / c) ** (2 / (g - 1)), uu, p * (cc / c) ** (2 * g / (g - 1))

    def cell_averages(self, xlo, xhi, n, x0, t, sub=400):
        """averages of (rho, rho u, E) over n equal cells of [xlo, xhi] at time
        t, the discontinuity initially at x0 (midpoint rule on sub points)"""
        dx = (xhi - xlo) / n
        xs = xlo + (np.arange(n * sub) + 0.5) * (dx / sub)
        out = np.zeros((3, n * sub))
        for k, x in enumerate(xs):
            r, u, p = self.sample((x - x0) / t)
            out[:, k] = (r, r * u, p / (self.g - 1) + 0.5 * r * u * u)
        return out.reshape(3, n, sub).mean(axis=2)
