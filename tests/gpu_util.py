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
                     eps=cfg.eps, charwise=int(cfg.characteristic),
                     smoothness=int(cfg.smoothness), alpha_stage=int(cfg.alpha_stage))


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


def natural_scales(spec, st):
    """Scale of every (var, comp) plane of a state: max |u-bar| for averages;
    for derivative averages the larger of their own max and the range of the
    component's averages over one cell (range/dx in 1D, where v-bar is a
    mean of u_x; range in 2D, where v-bar and w-bar are scaled by the cell
    size).  Limited derivatives next to a jump are tiny in absolute terms,
    and rounding there is measured against this scale."""
    S = np.zeros((spec.nvar, spec.K))
    for c in range(spec.K):
        u = st[0, c]
        rng = float(u.max() - u.min())
        S[0, c] = np.abs(u).max()
        for v in range(1, spec.nvar):
            S[v, c] = max(np.abs(st[v, c]).max(), rng / (spec.dx if spec.dim == 1 else 1.0))
    return np.where(S > 0, S, 1.0)


def scaled_err(gpu, ref, scales):
    """max over planes of max |gpu - ref| / scale of the plane, the scale being
    the larger of the given one and the plane's own magnitude in ref (a
    derivative can grow by orders of magnitude in one step next to a jump)"""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    ax = tuple(range(2, r.ndim))
    d = np.abs(g - r).max(axis=ax)
    return float((d / np.maximum(scales, np.abs(r).max(axis=ax))).max())


def rhs_scales(spec, st, ax, ay):
    """Scale of L: the state scale times the largest rate alpha_x/dx (+
    alpha_y/dy) at which the scheme moves it."""
    rate = ax / spec.dx + (ay / spec.dy if spec.dim == 2 else 0.0)
    return natural_scales(spec, st) * max(rate, 1e-300)


def scaled_err_planes(gpu, ref, scales):
    """scaled_err per (var, comp) plane (array of shape (nvar, K))"""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    ax = tuple(range(2, r.ndim))
    d = np.abs(g - r).max(axis=ax)
    return d / np.maximum(scales, np.abs(r).max(axis=ax))


def oracle_sensitivity(fn, st, scales, rel=1e-15, samples=2, seed=0):
    """Per (var, comp) plane, the largest scaled distance between fn(st) and
    fn of st perturbed by a relative `rel` (normal noise), over a few draws:
    how far rounding-level input differences move the oracle's own result.
    Where the scheme amplifies them (strong jumps; in characteristic
    variables the projection with |L| |R| >> 1 at low sound speed), a GPU
    result that differs from the oracle only by rounding is held, plane by
    plane, to a bar of a few times this distance."""
    rng = np.random.default_rng(seed)
    ref = fn(st)
    worst = None
    for _ in range(samples):
        out = fn(st * (1.0 + rel * rng.standard_normal(st.shape)))
        e = scaled_err_planes(out, ref, scales)
        worst = e if worst is None else np.maximum(worst, e)
    return worst


def within_conditioning(gpu, ref, scales, sens, floor):
    """True if every plane's scaled error is at most max(floor, 10 * its
    oracle sensitivity); returns (ok, errors, bars) for the message"""
    err = scaled_err_planes(gpu, ref, scales)
    bar = np.maximum(floor, 10.0 * sens)
    return bool(np.all(err <= bar)), err, bar


def l1_scaled_planes(gpu, ref, scales):
    """mean |gpu - ref| over the cells of every (var, comp) plane, divided by
    the plane's scale (array of shape (nvar, K))"""
    g = np.asarray(gpu, dtype=np.float64)
    r = np.asarray(ref, dtype=np.float64)
    ax = tuple(range(2, r.ndim))
    return np.abs(g - r).mean(axis=ax) / scales


def l1_scaled(gpu, ref, scales):
    """worst plane of l1_scaled_planes: the L1 error of a result in units of
    each plane's natural scale"""
    return float(l1_scaled_planes(gpu, ref, scales).max())


def host_threads():
    """CPU threads this process may run on (the affinity mask, which a
    shared machine narrows below its core count)"""
    import os
    try:
        return max(1, len(os.sched_getaffinity(0)))
    except Exception:
        return os.cpu_count() or 1
