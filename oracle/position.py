"""Position marginalisation of the facet likelihood (oracle; test
infrastructure).

Sec. 2.4 marginalises the likelihood over the source position with a
uniform prior, partly analytically and by cross-correlation (its discussion
of unreliable fits names errors of that cross-correlation); the formulation
itself is in the cited methodology paper and is not restated.
The reading taken here:

  * a position offset x = (dl, dm) (radians, relative to the catalogue
    position) multiplies the facet model by exp(+2 pi i k.x), the sign of
    Eq. 1 (R1), so with flux marginalised as in likelihood.py

        D(x) = sum_c W_c f_c Re(Vbar_c exp(-2 pi i (uc_c dl + vc_c dm))),
        ln L(e, alpha, x) = D(x)^2 / (2 Mm) - ln(Mm) / 2,

    Mm being independent of x: D(x) is the cross-correlation of the facet
    data with the model at lag x (analytic in the flux, numerical over the
    position);
  * the uniform prior covers the square of side n_side * step centred on the
    catalogue position, and the integral over it is the mean over an
    n_side x n_side grid of offsets at spacing `step` (offsets (p1 - h) step
    along l and (p2 - h) step along m, h = (n_side - 1) / 2, offset index
    p = p1 * n_side + p2);
  * the scale length is marginalised afterwards exactly as without offsets:

        ln L(e) = ln sum_k w_k (1 / n_side^2) sum_p L(e, alpha_k, x_p).

n_side = 1 is the position-fixed likelihood of likelihood.py.
"""
from __future__ import annotations

import numpy as np

from .estimate import FLAG_EMPTY, Estimate, estimate
from .fit import Params
from .likelihood import alpha_knots, e_grid, log_alpha_weights
from .model import ARCSEC, shape_inv_t


def offset_grid(n_side, step_arcsec):
    """Offsets (dl, dm) in radians, [n_side^2] each, index p = p1 * n_side + p2."""
    if n_side < 1 or n_side % 2 != 1:
        raise ValueError("n_side must be odd and >= 1")
    h = (n_side - 1) // 2
    p1, p2 = np.meshgrid(np.arange(n_side), np.arange(n_side), indexing="ij")
    return ((p1.reshape(-1) - h) * step_arcsec * ARCSEC,
            (p2.reshape(-1) - h) * step_arcsec * ARCSEC)


def loglike_alpha_offsets(facet, e1, e2, alpha_arcsec, dl, dm, chunk=256):
    """ln L(e, alpha, x_p) for each (e1[j], e2[j]) and offset p: [n_points, n_off]."""
    e1 = np.atleast_1d(np.asarray(e1, dtype=np.float64))
    e2 = np.atleast_1d(np.asarray(e2, dtype=np.float64))
    alpha = alpha_arcsec * ARCSEC
    W = facet.wsum
    # cross-correlation data per (cell, offset): W Re(Vbar exp(-2 pi i k.x))
    phase = 2.0 * np.pi * (facet.uc[:, None] * np.asarray(dl)[None, :] + facet.vc[:, None] * np.asarray(dm)[None, :])
    G = W[:, None] * (facet.vbar[:, None] * np.exp(-1j * phase)).real          # [n_cells, n_off]
    out = np.empty((e1.shape[0], G.shape[1]))
    for j0 in range(0, e1.shape[0], chunk):
        a11, a12, a22 = shape_inv_t(e1[j0:j0 + chunk, None], e2[j0:j0 + chunk, None])
        ku = a11 * facet.uc[None, :] + a12 * facet.vc[None, :]
        kv = a12 * facet.uc[None, :] + a22 * facet.vc[None, :]
        f = (1.0 + 4.0 * np.pi ** 2 * alpha ** 2 * (ku * ku + kv * kv)) ** -1.5   # [chunk, n_cells]
        D = f @ G                                                              # [chunk, n_off]
        Mm = np.sum(W[None, :] * f * f, axis=1)
        out[j0:j0 + chunk] = D * D / (2.0 * Mm[:, None]) - 0.5 * np.log(Mm)[:, None]
    return out


def marginal_surface_pos(facet, e1, e2, knots, log_w, dl, dm):
    """ln L(e) marginalised over the offsets (mean) and the knots (weights w_k)."""
    L = np.stack([loglike_alpha_offsets(facet, e1, e2, a, dl, dm) for a in knots], axis=0)   # [k, j, p]
    L = L + np.asarray(log_w)[:, None, None]
    m = np.max(L, axis=(0, 2))
    return m + np.log(np.sum(np.exp(L - m[None, :, None]), axis=(0, 2)) / L.shape[2])


def fit_source_pos(facet, flux_jy, n_side, step_arcsec, p: Params = Params(), mu=None):
    """Full-grid surface and estimate (as fit.fit_source) of the
    position-marginalised likelihood."""
    i1, i2, e1, e2, valid = e_grid(p.n_e, p.e_step)
    surf = np.full(p.n_e * p.n_e, -np.inf)
    if facet.n_cells == 0:
        nan = float("nan")
        return surf, Estimate(nan, nan, nan, nan, nan, nan, -1, 0, FLAG_EMPTY)
    knots = alpha_knots(p.rmin, p.rmax, p.num_r)
    logw = log_alpha_weights(flux_jy, knots, p.add, p.esp, p.r_std, None if mu is None else [mu])[0]
    dl, dm = offset_grid(n_side, step_arcsec)
    surf[valid] = marginal_surface_pos(facet, e1[valid], e2[valid], knots, logw, dl, dm)
    return surf, estimate(surf, e1, e2, valid, p.n_e, p.frac, p.bad_sigma, p.bad_sqrtdet)
