"""Shape estimate from the likelihood surface (oracle; test infrastructure).

Sec. 2.4: the ellipticity measurement is the mean and standard deviation of
the ellipticity samples whose likelihood is above 5 % of the maximum.  The
samples here are the full grid (the adaptive sampler is not on this path).
Reading R13: the moments are likelihood-weighted over the thresholded set,
in the population (1/sum w) form.  Sec. 2.4 and 4.1: a fit is bad when an
ellipticity standard deviation, or the square root of the covariance
determinant, is too small (defaults 5e-3 and 5e-5).
"""
from __future__ import annotations

import dataclasses
import math

import numpy as np

FLAG_BAD_VAR = 1      # variance too small to be realistic
FLAG_EMPTY = 2        # facet holds no visibility
FLAG_EDGE = 4         # maximum on the edge of the ellipticity domain
FLAG_FALLBACK = 8     # narrowed grid rejected, full grid used


@dataclasses.dataclass
class Estimate:
    e1: float
    e2: float
    s1: float
    s2: float
    c12: float
    lmax: float
    argmax: int
    n_above: int
    flags: int


def _edge(idx, n_e, valid):
    i1, i2 = divmod(idx, n_e)
    if i1 in (0, n_e - 1) or i2 in (0, n_e - 1):
        return True
    for d1, d2 in ((1, 0), (-1, 0), (0, 1), (0, -1)):
        if not valid[(i1 + d1) * n_e + (i2 + d2)]:
            return True
    return False


def estimate(surface, e1, e2, valid, n_e, frac=0.05, bad_sigma=5e-3, bad_sqrtdet=5e-5):
    """Thresholded likelihood-weighted moments of the surface.

    surface, e1, e2, valid: flattened [n_e*n_e] with i1 (e1) slow.  The
    maximum takes the smallest flat index among equal values.  The set is
    {e : l(e) >= l_max + ln frac}, weights exp(l - l_max).
    """
    s = np.where(valid, surface, -np.inf)
    idx = int(np.argmax(s))
    lmax = float(s[idx])
    if not np.isfinite(lmax):
        nan = float("nan")
        return Estimate(nan, nan, nan, nan, nan, nan, -1, 0, FLAG_EMPTY)
    above = valid & (s >= lmax + math.log(frac))
    wgt = np.exp(s[above] - lmax)
    x1, x2 = e1[above], e2[above]
    tw = np.sum(wgt)
    m1 = np.sum(wgt * x1) / tw
    m2 = np.sum(wgt * x2) / tw
    c11 = np.sum(wgt * (x1 - m1) ** 2) / tw
    c22 = np.sum(wgt * (x2 - m2) ** 2) / tw
    c12 = np.sum(wgt * (x1 - m1) * (x2 - m2)) / tw
    s1, s2 = math.sqrt(c11), math.sqrt(c22)
    det = c11 * c22 - c12 * c12
    sqrtdet = math.sqrt(det) if det > 0 else 0.0
    flags = 0
    if s1 <= bad_sigma or s2 <= bad_sigma or sqrtdet <= bad_sqrtdet:
        flags |= FLAG_BAD_VAR
    if _edge(idx, n_e, valid):
        flags |= FLAG_EDGE
    return Estimate(float(m1), float(m2), s1, s2, float(c12), lmax, idx, int(np.count_nonzero(above)), flags)
