"""Sequential sky-model refinement around the hot path (oracle; test
infrastructure).

The paper's driver (Sec. 2.1, 2.3, 2.4, 3.1): sources are processed in
catalogue order (decreasing flux), the sky model starts from the
catalogue's shapes (circular), and after a source is fitted its measured
ellipticity replaces the model's, so later sources are extracted from data
with better-subtracted neighbours.  With several sources fitted at once
(chunks of C sources, as the paper's MPI tasks do) the model is updated
after each chunk; C = 1 is the serial code, C = N the data-parallel pass.
Sources whose fit is flagged as bad keep their previous model and are
fitted once more at the end against the final sky model.

Steps here follow that description literally: the residual of every chunk
is the data minus the full sky model recomputed from the current shapes.
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .estimate import FLAG_BAD_VAR, FLAG_EMPTY
from .extract import extract_facet, facet_theta
from .fit import Params, fit_source
from .model import sky_model

FLAG_REFIT = 16     # fitted again at the end against the final sky model


@dataclasses.dataclass
class SkyCatalogue:
    l: np.ndarray
    m: np.ndarray
    flux_jy: np.ndarray
    alpha_arcsec: np.ndarray
    e1: np.ndarray
    e2: np.ndarray


def _fit_one(o, resid, cur, s, p, mu):
    src = (cur.l[s], cur.m[s], cur.flux_jy[s], cur.alpha_arcsec[s], cur.e1[s], cur.e2[s])
    fac = extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, o.weight, resid, src,
                        facet_theta(cur.alpha_arcsec[s], p.K), p.ref_freq_hz, p.beta)
    return fit_source(fac, cur.flux_jy[s], p, None if mu is None else mu[s])


def fit_sequential(o, vis, cat, chunk, refit_bad=True, p: Params = Params(), mu=None):
    """o: observation (u_m, v_m, w_m, freq_hz, weight); vis: data [rows*chan];
    cat: catalogue (l, m, flux_jy, alpha_arcsec, e1, e2 = initial model
    shapes), in processing order.  Returns (estimates [n], final e1, e2)."""
    n = len(cat.l)
    cur = SkyCatalogue(*(np.array(getattr(cat, k), dtype=np.float64) for k in
                         ("l", "m", "flux_jy", "alpha_arcsec", "e1", "e2")))
    out = [None] * n
    for c0 in range(0, n, chunk):
        resid = vis - sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cur, p.ref_freq_hz, p.beta)
        idx = range(c0, min(n, c0 + chunk))
        for s in idx:
            out[s] = _fit_one(o, resid, cur, s, p, mu)[1]
        for s in idx:                            # the chunk's good fits refine the model
            if not out[s].flags & (FLAG_BAD_VAR | FLAG_EMPTY):
                cur.e1[s], cur.e2[s] = out[s].e1, out[s].e2
    if refit_bad:
        bad = [s for s in range(n) if out[s].flags & FLAG_BAD_VAR]
        if bad:
            resid = vis - sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cur, p.ref_freq_hz, p.beta)
            for s in bad:
                est = _fit_one(o, resid, cur, s, p, mu)[1]
                out[s] = dataclasses.replace(est, flags=est.flags | FLAG_REFIT)
            for s in bad:
                if np.isfinite(out[s].e1):
                    cur.e1[s], cur.e2[s] = out[s].e1, out[s].e2
    return out, cur.e1, cur.e2
