"""Exponential-disk visibility model and sky model (oracle; test infrastructure).

Follows Sec. 2.2 of the paper: Eq. 1 (visibility of a sheared exponential
disk with a w-term), Eq. 2 (shear matrix A), Eq. 3 (ellipticity definition)
and Eq. 4 (median scale length from flux).
"""
from __future__ import annotations

import numpy as np

ARCSEC = np.pi / 648000.0          # radians per arcsecond
C_LIGHT = 299792458.0              # m/s


def wavelengths(x_m, freq_hz):
    """Baseline coordinate in wavelengths, shape [n_rows, n_chan].

    Sec. 2.2: (u, v, w) are measured in wavelengths at each channel centre.
    Two roundings: s_c = nu_c / c, then x = x_m * s_c.
    """
    s = np.asarray(freq_hz, dtype=np.float64) / C_LIGHT
    return np.asarray(x_m, dtype=np.float64)[:, None] * s[None, :]


def spectral_factor(freq_hz, ref_freq_hz, beta):
    """(lambda_ref / lambda)^beta of Eq. 1, i.e. (nu / nu_ref)^beta."""
    return (np.asarray(freq_hz, dtype=np.float64) / ref_freq_hz) ** beta


def n_minus_one(l, m):
    """sqrt(1 - l^2 - m^2) - 1 of Eq. 1, in the cancellation-free form."""
    r2 = l * l + m * m
    return -r2 / (1.0 + np.sqrt(1.0 - r2))


def shape_inv_t(e1, e2):
    """A^{-T} for the shear matrix A = [[1-e1, -e2], [-e2, 1+e1]] of Eq. 2.

    A is symmetric, so A^{-T} = A^{-1} = [[1+e1, e2], [e2, 1-e1]] / det A with
    det A = 1 - e1^2 - e2^2.  Returned as (a11, a12, a22).
    """
    det = 1.0 - e1 * e1 - e2 * e2
    return (1.0 + e1) / det, e2 / det, (1.0 - e1) / det


def disk_profile(u, v, alpha_arcsec, e1, e2):
    """Shape factor of Eq. 1: (1 + 4 pi^2 alpha^2 |A^{-T} k|^2)^{-3/2}, k = (u, v)."""
    a11, a12, a22 = shape_inv_t(e1, e2)
    ku = a11 * u + a12 * v
    kv = a12 * u + a22 * v
    alpha = alpha_arcsec * ARCSEC
    return (1.0 + 4.0 * np.pi ** 2 * alpha ** 2 * (ku * ku + kv * kv)) ** -1.5


def disk_vis(u, v, w, l, m, flux, alpha_arcsec, e1, e2, spec=1.0):
    """Eq. 1: visibility of one exponential disk at (u, v, w) in wavelengths.

    V = spec * S * exp(+2 pi i (u l + v m + w (sqrt(1-l^2-m^2) - 1))) * profile.
    The sign of the exponent is the paper's (reading R1).
    """
    phase = u * l + v * m + w * n_minus_one(l, m)
    return spec * flux * disk_profile(u, v, alpha_arcsec, e1, e2) * np.exp(2j * np.pi * phase)


def sky_model(u_m, v_m, w_m, freq_hz, cat, ref_freq_hz=1.4e9, beta=-0.7, sources=None):
    """Sec. 2.2: the sky model is the sum over catalogue sources of Eq. 1.

    Returns complex128 [n_rows * n_chan], channel fastest.  `cat` has arrays
    l, m, flux_jy, alpha_arcsec, e1, e2; `sources` restricts the sum.
    """
    u = wavelengths(u_m, freq_hz)
    v = wavelengths(v_m, freq_hz)
    w = wavelengths(w_m, freq_hz)
    spec = spectral_factor(freq_hz, ref_freq_hz, beta)[None, :]
    out = np.zeros(u.shape, dtype=np.complex128)
    idx = range(len(cat.l)) if sources is None else sources
    for s in idx:
        out += disk_vis(u, v, w, cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s],
                        cat.e1[s], cat.e2[s], spec)
    return out.reshape(-1)


def alpha_from_flux(flux_jy, add=-0.93, esp=0.33):
    """Eq. 4: ln(alpha_med / arcsec) = ADD + ESP ln(S / uJy)."""
    return np.exp(add + esp * np.log(np.asarray(flux_jy, dtype=np.float64) * 1e6))
