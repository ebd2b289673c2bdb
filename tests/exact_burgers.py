"""Exact cell averages of the smooth Burgers examples (Sec. 3.1, Examples 1
and 3) before shocks form: test infrastructure for the accuracy tables."""
import numpy as np


def burgers1d_exact_avg(nx, t, nq=10):
    """Example 1: cell averages of the exact solution on [0, 2] at time t
    (characteristics solved by Newton, Gauss rule per cell)"""
    dx = 2.0 / nx
    g, w = np.polynomial.legendre.leggauss(nq)
    g, w = 0.5 * (g + 1), 0.5 * w
    avg = np.zeros(nx)
    for gq, wq in zip(g, w):
        x = dx * (np.arange(nx) + gq)
        xi = x.copy()
        for _ in range(80):   # characteristics: x = xi + u0(xi) t
            xi -= (xi + (0.5 + np.sin(np.pi * xi)) * t - x) / (1 + np.pi * np.cos(np.pi * xi) * t)
        avg += wq * (0.5 + np.sin(np.pi * xi))
    return avg


def burgers2d_exact_avg(n, t, nq=6):
    """Example 3: cell averages of the exact solution on [0, 4]^2 at time t
    (u depends on x + y; characteristics solved by Newton)"""
    dx = 4.0 / n
    g, w = np.polynomial.legendre.leggauss(nq)
    g, w = 0.5 * (g + 1), 0.5 * w
    J, I = np.meshgrid(np.arange(n), np.arange(n), indexing="ij")
    avg = np.zeros((n, n))
    for a in range(nq):
        for b in range(nq):
            s = (I + g[a]) * dx + (J + g[b]) * dx
            xi = s.copy()
            for _ in range(60):   # u = u0(s - 2 u t), s = x + y
                xi -= (xi + 2 * (0.5 + np.sin(0.5 * np.pi * xi)) * t - s) / \
                      (1 + np.pi * np.cos(0.5 * np.pi * xi) * t)
            avg += w[a] * w[b] * (0.5 + np.sin(0.5 * np.pi * xi))
    return avg
