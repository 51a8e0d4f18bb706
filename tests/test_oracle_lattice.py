"""Pins of the lattice-seeded window (oracle.fit.lattice_window and
lattice_narrowed_fit; a narrowing of the grid that is not in the paper):
hand-worked boxes, a brute-force reading of the definition on random
surfaces, and the narrowed fit equal to the full-grid fit on real facets."""
import math

import numpy as np
import pytest

import oracle
from oracle.estimate import FLAG_FALLBACK
from paper_2203_14071_amd import synth

P = oracle.Params()


def _surface(points):
    """ln L = 0 at the given (i1, i2) grid points, -100 elsewhere (valid points only)."""
    i1, i2, _, _, valid = oracle.e_grid(P.n_e, P.e_step)
    s = np.where(valid, -100.0, -np.inf)
    for a, b in points:
        s[a * P.n_e + b] = 0.0
    return s


def test_hand_worked_boxes():
    # lattice points (40 + 4 q): members at (44, 36) and (52, 40): box widened by 4
    assert oracle.lattice_window(_surface([(44, 36), (52, 40)]), 4, P) == (40, 56, 32, 44)
    # a member of the rim lattice is clamped to the grid
    assert oracle.lattice_window(_surface([(0, 40), (4, 44)]), 4, P) == (0, 8, 36, 48)
    # off-lattice values are not read
    assert oracle.lattice_window(_surface([(44, 36), (53, 41)]), 4, P) == (40, 48, 32, 40)
    # stride 3: lattice 40 + 3 q
    assert oracle.lattice_window(_surface([(43, 37)]), 3, P) == (40, 46, 34, 40)
    # nothing finite on the lattice
    i1, i2, _, _, valid = oracle.e_grid(P.n_e, P.e_step)
    assert oracle.lattice_window(np.full(P.n_e * P.n_e, -np.inf), 4, P) is None


@pytest.mark.parametrize("seed", range(20))
def test_brute_force_reading(seed):
    g = np.random.default_rng(seed)
    i1, i2, _, _, valid = oracle.e_grid(P.n_e, P.e_step)
    c1, c2 = g.uniform(10, 70, 2)
    w = g.uniform(2, 15)
    surf = np.where(valid, -((i1 - c1) ** 2 + (i2 - c2) ** 2) / (2 * w * w) + g.normal(0, 0.3, i1.size), -np.inf)
    S = int(g.integers(2, 6))
    # the definition, point by point
    best = -math.inf
    for a in range(P.n_e):
        for b in range(P.n_e):
            if (a - 40) % S == 0 and (b - 40) % S == 0 and (a - 40) ** 2 + (b - 40) ** 2 < 2500:
                best = max(best, surf[a * P.n_e + b])
    lo1 = lo2 = 10 ** 9
    hi1 = hi2 = -1
    for a in range(P.n_e):
        for b in range(P.n_e):
            if (a - 40) % S == 0 and (b - 40) % S == 0 and (a - 40) ** 2 + (b - 40) ** 2 < 2500:
                if surf[a * P.n_e + b] >= best + math.log(0.05):
                    lo1, hi1, lo2, hi2 = min(lo1, a), max(hi1, a), min(lo2, b), max(hi2, b)
    want = (max(lo1 - S, 0), min(hi1 + S, 80), max(lo2 - S, 0), min(hi2 + S, 80))
    assert oracle.lattice_window(surf, S, P) == want


def test_narrowed_fit_equals_full_grid_on_real_facets():
    cfg = synth.small_config(0, n_ant=14, n_time=24, n_src=4)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(8))
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    rng = np.random.default_rng(9)
    vis = vis + 0.3 * cfg.noise_sigma_jy * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    kept = 0
    for s in range(cat.n_src):
        src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], cat.e1[s], cat.e2[s])
        fac = oracle.extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, o.weight, resid, src,
                                   oracle.facet_theta(cat.alpha_arcsec[s]))
        _, full = oracle.fit_source(fac, cat.flux_jy[s], P)
        _, est, refit = oracle.lattice_narrowed_fit(fac, cat.flux_jy[s], 4, P)
        if refit:
            assert est.flags & FLAG_FALLBACK
            assert (est.e1, est.e2) == (full.e1, full.e2)
            continue
        kept += 1
        # the window holds the whole thresholded set: the same estimate
        assert est.argmax == full.argmax and est.n_above == full.n_above
        assert est.e1 == pytest.approx(full.e1, abs=1e-12) and est.e2 == pytest.approx(full.e2, abs=1e-12)
        assert est.s1 == pytest.approx(full.s1, abs=1e-12) and est.s2 == pytest.approx(full.s2, abs=1e-12)
    assert kept >= 2
