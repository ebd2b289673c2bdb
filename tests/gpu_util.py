"""Shared helpers of the GPU tests: oracle problems for workload specs and
the parity measures used by every comparison."""
import numpy as np

import oracle as O


def oproblem(spec, cfg):
    """Oracle problem equal to a workload spec run with a library config."""
    return O.Problem(dim=spec.dim, flux=spec.flux, nx=spec.nx, ny=spec.ny, xlo=spec.xlo,
                     xhi=spec.xhi, ylo=spec.ylo, yhi=spec.yhi, bc_x=spec.bc_x, bc_y=spec.bc_y,
                     gas_gamma=spec.gas_gamma, adv=tuple(spec.adv), gauss_q=cfg.gauss_q,
                     weights=cfg.weights, gamma_lin=tuple(cfg.gamma_lin)[:3 if spec.dim == 1 else 5],
                     eps=cfg.eps)


def plane_rel(gpu, ref):
    """max over (var, comp) planes of max|gpu - ref| / max|ref| of the plane
    (a plane that is identically zero in the reference is measured against 1)."""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    ax = tuple(range(2, r.ndim))
    scale = np.abs(r).max(axis=ax, keepdims=True)
    scale = np.where(scale > 0, scale, 1.0)
    return float((np.abs(g - r) / scale).max())


def l1_rel(gpu, ref):
    """mean |gpu - ref| over the cells, relative to the mean |ref|, worst plane"""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    ax = tuple(range(2, r.ndim))
    den = np.abs(r).mean(axis=ax)
    den = np.where(den > 0, den, 1.0)
    return float((np.abs(g - r).mean(axis=ax) / den).max())
