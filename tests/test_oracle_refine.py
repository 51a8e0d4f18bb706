"""Pins of the adaptive refinement oracle (Sec. 2.4: samples around the
maximum until NP_MAX above the threshold or resolution E_RES)."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle.refine import FLAG_REFINED, _next_window, last_level, refine_source


def _sharp_facet(e1, e2, weight=1e14):
    """uv samples on cell centres, alpha on a knot, noiseless: the
    likelihood peaks exactly at the injected shape (as in P11)."""
    p = oracle.Params(num_r=8)
    alpha = oracle.alpha_knots(p.rmin, p.rmax, p.num_r)[4]
    theta = oracle.facet_theta(alpha)
    g = np.arange(-14, 15)
    IX, IY = np.meshgrid(g, g, indexing="ij")
    u, v = IX.reshape(-1) / theta, IY.reshape(-1) / theta
    data = 2e-4 * oracle.model.disk_profile(u, v, alpha, e1, e2) + 0j
    n = u.shape[0]
    f = oracle.extract_facet(u, v, np.zeros(n), np.array([299792458.0]), np.full(n, weight), data,
                             (0.0, 0.0, 0.0, alpha, 0.0, 0.0), theta)
    return f, p, math.log(alpha)


def test_levels_and_windows():
    assert last_level(0.02, 0.003) == 3            # 0.01, 0.005, 0.0025
    assert last_level(0.02, 0.005) == 2 and last_level(0.02, 0.02) == 0 and last_level(0.02, 0.019) == 1
    assert _next_window(3, 5, 4) == (4, 12)          # [2*3-2, 2*5+2]
    assert _next_window(-40, 40, 7) == (14 - 31, 14 - 31 + 63)   # too wide: 64 points around the maximum


def test_refinement_resolves_an_off_grid_peak():
    """Injected shape on the level-3 lattice (k * 0.0025) between coarse
    points: the coarse set is a single point off the truth; the refined
    estimate lands on the truth."""
    e1, e2 = 123 * (0.02 / 8), -45 * (0.02 / 8)      # 0.3075, -0.1125
    f, p, mu = _sharp_facet(e1, e2)
    surf, est = oracle.fit_source(f, 2e-4, p, mu=mu)
    assert est.n_above < 30 and math.hypot(est.e1 - e1, est.e2 - e2) > 5e-3
    ref = refine_source(f, 2e-4, surf, est, p, mu=mu)
    assert ref.flags & FLAG_REFINED
    assert ref.e1 == pytest.approx(e1, abs=1e-9) and ref.e2 == pytest.approx(e2, abs=1e-9)
    assert ref.lmax >= est.lmax


def test_refined_samples_on_coarse_points_equal_the_coarse_surface():
    """Level-1 lattice points with even k are coarse grid points: same e
    (a power-of-two step ratio), hence the same log-likelihood."""
    f, p, mu = _sharp_facet(0.1, 0.05, weight=1e6)
    knots = oracle.alpha_knots(p.rmin, p.rmax, p.num_r)
    logw = oracle.log_alpha_weights(2e-4, knots, p.add, p.esp, p.r_std, [mu])[0]
    k1, k2 = np.array([4, 6, -10]), np.array([6, -2, 0])        # even level-1 indices
    fine = oracle.marginal_surface(f, k1 * (p.e_step / 2), k2 * (p.e_step / 2), knots, logw)
    coarse = oracle.marginal_surface(f, (k1 // 2) * p.e_step, (k2 // 2) * p.e_step, knots, logw)
    assert np.array_equal(fine, coarse)


def test_broad_posteriors_are_left_alone():
    f, p, mu = _sharp_facet(0.2, -0.1, weight=1e-1)  # low signal-to-noise: a wide set
    surf, est = oracle.fit_source(f, 2e-4, p, mu=mu)
    assert est.n_above >= 30
    assert refine_source(f, 2e-4, surf, est, p, mu=mu) is est


def test_refined_widths_clear_the_grid_limited_bad_flag():
    """A peak narrower than the coarse step is flagged BAD_VAR on the coarse
    grid (R18); moderately sharp data refined to 0.0025 resolve a width
    above the threshold and drop the flag."""
    e1, e2 = 0.2, 0.1
    for w in (3e9, 1e10, 3e10):
        f, p, mu = _sharp_facet(e1, e2, weight=w)
        surf, est = oracle.fit_source(f, 2e-4, p, mu=mu)
        ref = refine_source(f, 2e-4, surf, est, p, mu=mu)
        if est.flags & oracle.FLAG_BAD_VAR and not ref.flags & oracle.FLAG_BAD_VAR:
            assert ref.s1 > p.bad_sigma and ref.s2 > p.bad_sigma and ref.n_above > est.n_above
            return
    pytest.fail("no weight gave a grid-limited coarse fit that refinement resolves")
