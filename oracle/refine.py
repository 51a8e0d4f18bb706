"""Adaptive refinement of the ellipticity estimate (oracle; test
infrastructure).

Sec. 2.4 samples the likelihood adaptively around its maximum until either
NP_MAX = 30 samples lie above the 5 % threshold or the resolution E_RES =
0.003 is reached, and takes the mean and standard deviation of the samples
above the threshold.  Here the adaptive sampler is a nested grid: level L
has the points e = k * step / 2^L (k integer, |e| < 1 tested on the
integers), level 0 being the full grid of the fit.  A source whose
thresholded set at level L holds fewer than NP_MAX points is sampled at
level L + 1 on a window covering that set's bounding box widened by one
level-L step on every side (at most MAX_SIDE points per axis, else centred
on the maximum); the last level is the first whose step is <= E_RES.  The
estimate is the thresholded, likelihood-weighted mean and covariance of the
last level's window (as in estimate.py), flagged REFINED; the bad-variance
flag is re-evaluated with the refined widths.
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

from .estimate import FLAG_BAD_VAR, FLAG_EMPTY
from .fit import Params
from .likelihood import alpha_knots, e_grid, log_alpha_weights, marginal_surface
from .position import marginal_surface_pos, offset_grid

FLAG_REFINED = 32
MAX_SIDE = 64


def last_level(e_step, e_res):
    """Smallest L >= 1 with e_step / 2^L <= e_res (0: no refinement)."""
    if e_step <= e_res:
        return 0
    L = 1
    while e_step / 2.0 ** L > e_res:
        L += 1
    return L


def _next_window(kmin, kmax, karg, max_side=MAX_SIDE):
    """Integer range at the next level covering [kmin, kmax] widened by one
    current step, or max_side points centred on karg."""
    lo, hi = 2 * kmin - 2, 2 * kmax + 2
    if hi - lo + 1 > max_side:
        lo = 2 * karg - (max_side - 1) // 2
        hi = lo + max_side - 1
    return lo, hi


def _scan(values, k1, k2, frac):
    """Maximum (first on ties), thresholded members and their bounding box."""
    fin = np.isfinite(values)
    j = int(np.argmax(np.where(fin, values, -np.inf)))
    lmax = float(values[j])
    member = fin & (values >= lmax + math.log(frac))
    return j, lmax, member


def refine_source(facet, flux_jy, surface, est, p: Params = Params(), np_max=30, e_res=0.003, mu=None,
                  position=None):
    """surface, est: the full-grid fit of this facet (fit_source, or
    position.fit_source_pos with position = (n_side, step_arcsec), whose
    position-marginalised likelihood the finer levels then use as well).
    Returns the refined estimate (or est itself when no refinement is
    needed)."""
    if est.flags & FLAG_EMPTY:
        return est
    i1, i2, _, _, valid = e_grid(p.n_e, p.e_step)
    c = (p.n_e - 1) // 2
    vals = np.where(valid, surface, -np.inf)
    j, lmax, member = _scan(vals, i1 - c, i2 - c, p.frac)
    count = int(np.count_nonzero(member))
    Lmax = last_level(p.e_step, e_res)
    if count >= np_max or Lmax == 0:
        return est
    unit = int(round(1.0 / p.e_step))
    knots = alpha_knots(p.rmin, p.rmax, p.num_r)
    logw = log_alpha_weights(flux_jy, knots, p.add, p.esp, p.r_std, None if mu is None else [mu])[0]
    k1m, k2m = (i1 - c)[member], (i2 - c)[member]
    w1 = _next_window(int(k1m.min()), int(k1m.max()), int(i1[j] - c))
    w2 = _next_window(int(k2m.min()), int(k2m.max()), int(i2[j] - c))
    L = 1
    while True:
        res = p.e_step / float(1 << L)
        K1, K2 = np.meshgrid(np.arange(w1[0], w1[1] + 1), np.arange(w2[0], w2[1] + 1), indexing="ij")
        K1, K2 = K1.reshape(-1), K2.reshape(-1)
        ok = K1.astype(np.int64) ** 2 + K2.astype(np.int64) ** 2 < (unit << L) ** 2
        e1, e2 = K1 * res, K2 * res
        vals = np.full(K1.shape, -np.inf)
        if np.any(ok):
            if position is None:
                vals[ok] = marginal_surface(facet, e1[ok], e2[ok], knots, logw)
            else:
                dl, dm = offset_grid(*position)
                vals[ok] = marginal_surface_pos(facet, e1[ok], e2[ok], knots, logw, dl, dm)
        j, lmax, member = _scan(vals, K1, K2, p.frac)
        count = int(np.count_nonzero(member))
        wgt = np.exp(vals[member] - lmax)
        sw = wgt.sum()
        m1, m2 = (wgt * e1[member]).sum() / sw, (wgt * e2[member]).sum() / sw
        d1, d2 = e1[member] - m1, e2[member] - m2
        c11, c22, c12 = (wgt * d1 * d1).sum() / sw, (wgt * d2 * d2).sum() / sw, (wgt * d1 * d2).sum() / sw
        s1, s2 = math.sqrt(c11), math.sqrt(c22)
        det = c11 * c22 - c12 * c12
        sqd = math.sqrt(det) if det > 0 else 0.0
        bad = s1 <= p.bad_sigma or s2 <= p.bad_sigma or sqd <= p.bad_sqrtdet
        flags = (est.flags & ~FLAG_BAD_VAR) | (FLAG_BAD_VAR if bad else 0) | FLAG_REFINED
        out = dataclasses.replace(est, e1=float(m1), e2=float(m2), s1=s1, s2=s2, c12=float(c12), lmax=lmax,
                                  n_above=count, flags=flags)
        if count >= np_max or L == Lmax:
            return out
        k1m, k2m = K1[member], K2[member]
        w1 = _next_window(int(k1m.min()), int(k1m.max()), int(K1[j]))
        w2 = _next_window(int(k2m.min()), int(k2m.max()), int(K2[j]))
        L += 1
