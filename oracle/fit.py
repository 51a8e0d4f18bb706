"""Per-source fit on a facet: surface over the full e-grid, then the estimate
(oracle; test infrastructure).  Sec. 2.4 of the paper, with the full grid in
place of the simplex maximiser and the adaptive sampler.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .estimate import FLAG_EMPTY, FLAG_FALLBACK, Estimate, estimate
from .likelihood import alpha_knots, e_grid, log_alpha_weights, marginal_surface


@dataclasses.dataclass(frozen=True)
class Params:
    """Algorithm parameters (Sec. 2: beta, ADD, ESP, PSF_NAT=K, RMIN, RMAX,
    NUM_R, R_STD; Sec. 4.1: K = 38 and the bad-fit thresholds)."""
    beta: float = -0.7
    ref_freq_hz: float = 1.4e9
    K: float = 38.0
    add: float = -0.93
    esp: float = 0.33
    r_std: float = 0.3136
    rmin: float = 0.3
    rmax: float = 3.5
    num_r: int = 20
    n_e: int = 81
    e_step: float = 0.02
    frac: float = 0.05
    bad_sigma: float = 5e-3
    bad_sqrtdet: float = 5e-5


def fit_source(facet, flux_jy, p: Params = Params(), mu=None, window=None):
    """Surface (flattened [n_e*n_e], -inf where masked or outside `window`)
    and the estimate for one facet.

    window: optional (i1lo, i1hi, i2lo, i2hi), inclusive, restricting the
    evaluated e-points.
    """
    i1, i2, e1, e2, valid = e_grid(p.n_e, p.e_step)
    if window is not None:
        a, b, c, d = window
        valid = valid & (i1 >= a) & (i1 <= b) & (i2 >= c) & (i2 <= d)
    surf = np.full(p.n_e * p.n_e, -np.inf)
    if facet.n_cells == 0:
        nan = float("nan")
        return surf, Estimate(nan, nan, nan, nan, nan, nan, -1, 0, FLAG_EMPTY)
    knots = alpha_knots(p.rmin, p.rmax, p.num_r)
    logw = log_alpha_weights(flux_jy, knots, p.add, p.esp, p.r_std,
                             None if mu is None else [mu])[0]
    surf[valid] = marginal_surface(facet, e1[valid], e2[valid], knots, logw)
    est = estimate(surf, e1, e2, valid, p.n_e, p.frac, p.bad_sigma, p.bad_sqrtdet)
    return surf, est


def window_rejected(surface, window, check_stride=0, p: Params = Params()):
    """The rule by which a narrowed fit distrusts its window (not in the
    paper).  surface: flattened [n_e*n_e] ln L(e), read inside the window and,
    with check_stride S > 0, at the lattice points outside it.  The window is
    rejected when
      * it holds no valid grid point (|e| < 1), or
      * a member of its thresholded set {ln L >= ln Lmax_w + ln frac} (Lmax_w
        the maximum inside the window) has one of its four grid neighbours
        valid but outside the window (the set, or the maximum, may continue
        beyond the window), or
      * S > 0 and a valid point outside the window whose offsets (i1 - c,
        i2 - c) from the grid centre are both multiples of S reaches that set
        (a separate region of high likelihood)."""
    i1, i2, _, _, valid = e_grid(p.n_e, p.e_step)
    a, b, c, d = window
    inside = (i1 >= a) & (i1 <= b) & (i2 >= c) & (i2 <= d)
    win = valid & inside
    if not np.any(win):
        return True
    thr = float(np.max(surface[win])) + math.log(p.frac)
    member = (win & (surface >= thr)).reshape(p.n_e, p.n_e)
    out = np.zeros((p.n_e + 2, p.n_e + 2), dtype=bool)          # valid and outside, padded by one
    out[1:-1, 1:-1] = (valid & ~inside).reshape(p.n_e, p.n_e)
    for di, dj in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        if np.any(member & out[1 + di:p.n_e + 1 + di, 1 + dj:p.n_e + 1 + dj]):
            return True
    if check_stride > 0:
        ctr = (p.n_e - 1) // 2
        lat = valid & ~inside & ((i1 - ctr) % check_stride == 0) & ((i2 - ctr) % check_stride == 0)
        if np.any(surface[lat] >= thr):
            return True
    return False


def narrowed_fit(facet, flux_jy, window, check_stride=0, p: Params = Params(), mu=None):
    """Fit on an ellipticity window; where window_rejected holds for a
    non-empty facet, the full-grid fit replaces it, flagged FALLBACK.
    Returns (surface, estimate, refitted)."""
    surf, est = fit_source(facet, flux_jy, p, mu, window)
    if facet.n_cells == 0:
        return surf, est, False
    full, full_est = fit_source(facet, flux_jy, p, mu)
    seen = full.copy()                          # the window's own values inside it
    inw = np.isfinite(surf)
    seen[inw] = surf[inw]
    if not window_rejected(seen, window, check_stride, p):
        return surf, est, False
    return full, dataclasses.replace(full_est, flags=full_est.flags | FLAG_FALLBACK), True


def lattice_window(surface, check_stride, p: Params = Params()):
    """Window seeded by a coarse lattice (not in the paper): from the values
    of ln L(e) at the valid grid points whose offsets (i1 - c, i2 - c) from
    the grid centre are both multiples of the stride S, the bounding box of
    the lattice points within the 5 % threshold of the lattice maximum,
    widened by S grid steps on every side and clamped to the grid
    (i1lo, i1hi, i2lo, i2hi).  surface: flattened [n_e*n_e], read at the
    lattice points only.  None when no lattice value is finite."""
    i1, i2, _, _, valid = e_grid(p.n_e, p.e_step)
    c = (p.n_e - 1) // 2
    lat = valid & ((i1 - c) % check_stride == 0) & ((i2 - c) % check_stride == 0)
    vals = np.where(lat, surface, -np.inf)
    if not np.any(np.isfinite(vals)):
        return None
    member = lat & (vals >= np.max(vals) + math.log(p.frac))
    return (max(int(i1[member].min()) - check_stride, 0), min(int(i1[member].max()) + check_stride, p.n_e - 1),
            max(int(i2[member].min()) - check_stride, 0), min(int(i2[member].max()) + check_stride, p.n_e - 1))


def lattice_narrowed_fit(facet, flux_jy, check_stride, p: Params = Params(), mu=None):
    """The fit narrowed to the lattice-seeded window (lattice_window), with
    the window rule and the full-grid fallback of narrowed_fit.  The lattice
    values are those of the full surface (the same function at the same
    points).  Returns (surface, estimate, refitted)."""
    full, _ = fit_source(facet, flux_jy, p, mu)
    window = lattice_window(full, check_stride, p)
    if window is None:
        window = (0, p.n_e - 1, 0, p.n_e - 1)
    return narrowed_fit(facet, flux_jy, window, check_stride, p, mu)


def fit_sources(facets, flux_jy, p: Params = Params(), mu=None):
    out = []
    for k, f in enumerate(facets):
        out.append(fit_source(f, flux_jy[k], p, None if mu is None else mu[k]))
    return out
