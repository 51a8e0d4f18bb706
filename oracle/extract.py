"""Source extraction into a per-source facet (oracle; test infrastructure).

Follows Sec. 2.3 of the paper: subtract every other source's sky-model
visibilities, phase-shift to the source, average into a coarse square uv
grid whose field of view is K times the source scale length.

Readings taken where the paper is silent:
  * the sky model of all sources is built from the catalogue's current shape
    (circular at the start), and the source's own model is added back, so
    data - sum_{t != s} V_t = (data - Sky) + V_s (R15);
  * cells are centred on the uv origin: ix = rint(u * theta) with round-half-
    even, nothing is truncated (R4);
  * averaging is weighted by the visibility weights (R8); flagged
    visibilities (w <= 0) are skipped;
  * conjugate points are not added (R9).
"""
from __future__ import annotations

import dataclasses

import numpy as np

from .model import ARCSEC, disk_profile, n_minus_one, spectral_factor, wavelengths


@dataclasses.dataclass
class Facet:
    theta: float                # field of view in radians; cell size 1/theta wavelengths
    ix: np.ndarray              # int64 [n_cells], sorted by (iy, ix)
    iy: np.ndarray
    count: np.ndarray           # int64 visibilities per cell
    wsum: np.ndarray            # sum of weights per cell
    vbar: np.ndarray            # complex weighted mean of the shifted visibilities
    uc: np.ndarray              # cell centre u = ix / theta (wavelengths)
    vc: np.ndarray

    @property
    def n_cells(self) -> int:
        return int(self.ix.shape[0])


def facet_theta(alpha_arcsec, K=38.0):
    """Sec. 2.3: facet field of view theta = K * alpha (radians).

    alpha is converted to radians first, then multiplied by K.
    """
    return K * (alpha_arcsec * ARCSEC)


def extract_facet(u_m, v_m, w_m, freq_hz, weight, residual, src, theta,
                  ref_freq_hz=1.4e9, beta=-0.7):
    """Facet of one source.

    residual: data - Sky (all catalogue sources), complex [n_rows*n_chan],
    channel fastest.  src: (l, m, flux_jy, alpha_arcsec, e1, e2) of the
    source, whose own model is added back before the shift.
    """
    l, m, flux, alpha, e1, e2 = src
    u = wavelengths(u_m, freq_hz).reshape(-1)
    v = wavelengths(v_m, freq_hz).reshape(-1)
    w = wavelengths(w_m, freq_hz).reshape(-1)
    spec = np.broadcast_to(spectral_factor(freq_hz, ref_freq_hz, beta)[None, :],
                           (len(u_m), len(freq_hz))).reshape(-1)
    phase = u * l + v * m + w * n_minus_one(l, m)
    # own model after the shift is real: spec * S * profile (Eq. 1 times the shift)
    own = spec * flux * disk_profile(u, v, alpha, e1, e2)
    z = residual * np.exp(-2j * np.pi * phase) + own
    ix = np.rint(u * theta).astype(np.int64)
    iy = np.rint(v * theta).astype(np.int64)
    wt = np.asarray(weight, dtype=np.float64)
    keep = wt > 0
    ix, iy, wt, z = ix[keep], iy[keep], wt[keep], z[keep]
    if ix.size == 0:
        e = np.zeros(0, dtype=np.int64)
        return Facet(theta, e, e, e, np.zeros(0), np.zeros(0, np.complex128), np.zeros(0), np.zeros(0))
    # one integer key per (iy, ix) that sorts like the pair: iy major, ix minor
    x0, span = ix.min(), ix.max() - ix.min() + 1
    key = (iy - iy.min()) * span + (ix - x0)
    ukey, inv = np.unique(key, return_inverse=True)
    inv = inv.reshape(-1)
    count = np.bincount(inv).astype(np.int64)
    wsum = np.bincount(inv, weights=wt)
    zre = np.bincount(inv, weights=wt * z.real)
    zim = np.bincount(inv, weights=wt * z.imag)
    cy = ukey // span + iy.min()
    cx = ukey % span + x0
    return Facet(theta, cx, cy, count, wsum, (zre + 1j * zim) / wsum, cx / theta, cy / theta)


def extract_facets(u_m, v_m, w_m, freq_hz, weight, residual, cat, K=38.0, sources=None,
                   ref_freq_hz=1.4e9, beta=-0.7):
    """Facets of several catalogue sources (plain loop)."""
    idx = range(len(cat.l)) if sources is None else sources
    out = []
    for s in idx:
        theta = facet_theta(cat.alpha_arcsec[s], K)
        src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], cat.e1[s], cat.e2[s])
        out.append(extract_facet(u_m, v_m, w_m, freq_hz, weight, residual, src, theta,
                                 ref_freq_hz, beta))
    return out
