"""Facet likelihood, flux and scale-length marginalisation (oracle; test infrastructure).

Follows Sec. 2.4 of the paper.  The facet model is Eq. 1 with w = 0
evaluated at the cell centres (R10), it is real after the phase shift, and
the likelihood is chi-squared over the cells with the cell weight sums as
inverse variances (R8):

    chi2(S) = sum_c W_c |Vbar_c - S f_c|^2 .

Flux, under an improper uniform prior on the real line (R7), integrates in
closed form:

    ln int exp(-chi2/2) dS = D^2/(2 Mm) - ln(Mm)/2 + [ln(2 pi)/2 - sum_c W_c |Vbar_c|^2 / 2]

with D = sum_c W_c f_c Re Vbar_c and Mm = sum_c W_c f_c^2.  The bracket does
not depend on the shape parameters and is omitted.

Scale length is marginalised numerically over [RMIN, RMAX] on NUM_R knots
placed with quadratic spacing in the knot index (R5), with a log-normal prior
whose median follows Eq. 4 and whose width is R_STD (Sec. 2.4), using the
exact integral of the natural cubic spline through the knots (R6).  The
spline integral is linear in the knot values, so it reduces to fixed weights.
"""
from __future__ import annotations

import numpy as np

from .model import ARCSEC, shape_inv_t


def alpha_knots(rmin=0.3, rmax=3.5, n=20):
    """NUM_R scale-length knots, quadratic in the index: rmin + (rmax-rmin)(k/(n-1))^2."""
    t = np.arange(n, dtype=np.float64) / (n - 1)
    return rmin + (rmax - rmin) * t * t


def spline_quadrature_weights(x):
    """Weights c_k with int_{x_0}^{x_{n-1}} S(x) dx = sum_k c_k y_k for the
    natural cubic spline S through (x_k, y_k).

    With second derivatives M_k (M_0 = M_{n-1} = 0) solving the usual
    tridiagonal continuity system, each interval integrates to
    h (y_i + y_{i+1})/2 - h^3 (M_i + M_{i+1})/24.  Both terms are linear in y,
    so the weights are read off by applying the map to the identity.
    """
    x = np.asarray(x, dtype=np.float64)
    n = x.shape[0]
    h = np.diff(x)
    eye = np.eye(n)
    M = np.zeros((n, n))              # M = (second derivatives) as a linear map of y
    if n > 2:
        T = np.zeros((n - 2, n - 2))
        R = np.zeros((n - 2, n))
        for r, i in enumerate(range(1, n - 1)):
            T[r, r] = 2.0 * (h[i - 1] + h[i])
            if r > 0:
                T[r, r - 1] = h[i - 1]
            if r < n - 3:
                T[r, r + 1] = h[i]
            R[r] = 6.0 * ((eye[i + 1] - eye[i]) / h[i] - (eye[i] - eye[i - 1]) / h[i - 1])
        M[1:n - 1] = np.linalg.solve(T, R)
    c = np.zeros(n)
    for i in range(n - 1):
        c += h[i] * (eye[i] + eye[i + 1]) / 2.0 - h[i] ** 3 * (M[i] + M[i + 1]) / 24.0
    return c


def log_normal_prior(alpha, mu, sigma):
    """ln of the log-normal pdf in alpha (arcsec): median e^mu, width sigma in ln alpha."""
    alpha = np.asarray(alpha, dtype=np.float64)
    return -(np.log(alpha) - mu) ** 2 / (2.0 * sigma ** 2) - np.log(alpha * sigma * np.sqrt(2.0 * np.pi))


def log_alpha_weights(flux_jy, knots, add=-0.93, esp=0.33, r_std=0.3136, mu=None):
    """ln(c_k p_s(alpha_k)) per source: spline weight times prior at each knot.

    The prior median follows Eq. 4 unless `mu` (ln of the median in arcsec)
    is given per source.  Shape [n_src, n_knots].
    """
    flux_jy = np.atleast_1d(np.asarray(flux_jy, dtype=np.float64))
    if mu is None:
        mu = add + esp * np.log(flux_jy * 1e6)
    mu = np.atleast_1d(np.asarray(mu, dtype=np.float64))
    c = spline_quadrature_weights(knots)
    return np.log(c)[None, :] + log_normal_prior(knots[None, :], mu[:, None], r_std)


def e_grid(n_e=81, step=0.02):
    """Ellipticity grid e = (i - (n_e-1)/2) * step on both axes, i1 (e1) slow.

    A point is valid when |e| < 1, tested on the integers:
    (i1-c)^2 + (i2-c)^2 < (1/step)^2 with c = (n_e-1)/2 (R14).
    Returns (i1, i2, e1, e2, valid), each flattened [n_e*n_e].
    """
    R = int(round(1.0 / step))
    if n_e % 2 != 1 or abs(R * step - 1.0) > 1e-9:
        raise ValueError("n_e must be odd and 1/step an integer")
    c = (n_e - 1) // 2
    i1, i2 = np.meshgrid(np.arange(n_e), np.arange(n_e), indexing="ij")
    i1, i2 = i1.reshape(-1), i2.reshape(-1)
    valid = (i1 - c) ** 2 + (i2 - c) ** 2 < R * R
    return i1, i2, (i1 - c) * step, (i2 - c) * step, valid


def loglike_alpha(facet, e1, e2, alpha_arcsec, chunk=512):
    """ln L(e, alpha) = D^2/(2 Mm) - ln(Mm)/2 at each (e1[j], e2[j]) for one alpha.

    f_c = (1 + 4 pi^2 alpha^2 |A_e^{-T} k_c|^2)^{-3/2} at the cell centres k_c.
    """
    e1 = np.atleast_1d(np.asarray(e1, dtype=np.float64))
    e2 = np.atleast_1d(np.asarray(e2, dtype=np.float64))
    alpha = alpha_arcsec * ARCSEC
    out = np.empty(e1.shape[0])
    W = facet.wsum[None, :]
    vr = facet.vbar.real[None, :]
    for j0 in range(0, e1.shape[0], chunk):
        a11, a12, a22 = shape_inv_t(e1[j0:j0 + chunk, None], e2[j0:j0 + chunk, None])
        ku = a11 * facet.uc[None, :] + a12 * facet.vc[None, :]
        kv = a12 * facet.uc[None, :] + a22 * facet.vc[None, :]
        f = (1.0 + 4.0 * np.pi ** 2 * alpha ** 2 * (ku * ku + kv * kv)) ** -1.5
        D = np.sum(W * f * vr, axis=1)
        Mm = np.sum(W * f * f, axis=1)
        out[j0:j0 + chunk] = D * D / (2.0 * Mm) - 0.5 * np.log(Mm)
    return out


def marginal_surface(facet, e1, e2, knots, log_w):
    """ln of the scale-length-marginalised likelihood at each e:

        l(e) = m + ln sum_k exp(ln w_k + l(e, alpha_k) - m),  m = max_k l(e, alpha_k).
    """
    L = np.stack([loglike_alpha(facet, e1, e2, a) for a in knots], axis=0)   # [n_knots, n_e]
    m = np.max(L, axis=0)
    return m + np.log(np.sum(np.exp(np.asarray(log_w)[:, None] + L - m[None, :]), axis=0))
