"""Pins of the position-marginalisation oracle (Sec. 2.4; the reading is in
oracle/position.py): one offset is the position-fixed likelihood; for a
noiseless source displaced by a grid offset, with every visibility at a cell
centre, the cross-correlation at the true lag equals the flux times the
model energy (a closed form) and is the largest over the offsets; the
marginalised fit of a displaced source is the fit of the undisplaced one."""
import numpy as np
import pytest

import oracle
from oracle.model import ARCSEC, C_LIGHT, disk_profile
from oracle.sequential import SkyCatalogue
from paper_2203_14071_amd import synth

E_TRUE = (0.3, -0.2)
FLUX = 100e-6
STEP = 0.3                                        # arcsec between offsets


def _centred(q, n_side=5, seed=3, wscale=1e8):
    """Facet of a noiseless source displaced from its catalogue position by
    offset q = (p1, p2) of the n_side grid; one channel at nu = c (so u in
    wavelengths equals u in metres), w = 0, every visibility at a cell centre
    of the facet, 1 to 3 visibilities per cell, weights ~wscale."""
    rng = np.random.default_rng(seed)
    alpha = oracle.alpha_knots()[10]              # a knot, so the true size is on the quadrature
    theta = oracle.facet_theta(alpha)
    n = 14
    ix, iy = np.meshgrid(np.arange(-n, n + 1), np.arange(-n, n + 1), indexing="ij")
    ix, iy = ix.reshape(-1), iy.reshape(-1)
    keep = rng.random(ix.size) < 0.6
    ix, iy = ix[keep], iy[keep]
    rep = rng.integers(1, 4, ix.size)
    u, v = np.repeat(ix / theta, rep), np.repeat(iy / theta, rep)
    w = np.zeros_like(u)
    freq = np.array([C_LIGHT])
    wt = rng.uniform(0.5, 2.0, u.size) * wscale
    h = (n_side - 1) // 2
    dl, dm = (q[0] - h) * STEP * ARCSEC, (q[1] - h) * STEP * ARCSEC
    l0, m0 = 0.001, -0.0005

    def cat(l, m):
        return SkyCatalogue(np.array([l]), np.array([m]), np.array([FLUX]), np.array([alpha]),
                            np.array([E_TRUE[0]]), np.array([E_TRUE[1]]))

    resid = oracle.sky_model(u, v, w, freq, cat(l0 + dl, m0 + dm)) - oracle.sky_model(u, v, w, freq, cat(l0, m0))
    fac = oracle.extract_facet(u, v, w, freq, wt, resid, (l0, m0, FLUX, alpha, *E_TRUE), theta)
    spec = oracle.spectral_factor(freq, 1.4e9, -0.7)[0]
    return fac, alpha, spec


def test_offset_grid_layout():
    dl, dm = oracle.offset_grid(3, 0.5)
    assert dl.shape == dm.shape == (9,)
    # p = p1 * 3 + p2; p1 along l, p2 along m, centred
    assert (dl[5], dm[5]) == (0.0, 0.5 * ARCSEC)
    assert (dl[1], dm[1]) == (-0.5 * ARCSEC, 0.0)
    assert dl[4] == dm[4] == 0.0
    with pytest.raises(ValueError):
        oracle.offset_grid(4, 0.1)


def test_single_offset_is_the_position_fixed_likelihood():
    cfg = synth.small_config(0, n_ant=10, n_time=12, n_src=2)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(4))
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    rng = np.random.default_rng(5)
    vis = vis + cfg.noise_sigma_jy * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    src = (cat.l[0], cat.m[0], cat.flux_jy[0], cat.alpha_arcsec[0], cat.e1[0], cat.e2[0])
    fac = oracle.extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, o.weight, resid, src,
                               oracle.facet_theta(cat.alpha_arcsec[0]))
    p = oracle.Params()
    s0, e0 = oracle.fit_source(fac, cat.flux_jy[0], p)
    s1, e1 = oracle.fit_source_pos(fac, cat.flux_jy[0], 1, 0.3, p)
    fin = np.isfinite(s0)
    assert np.array_equal(fin, np.isfinite(s1))
    np.testing.assert_allclose(s1[fin], s0[fin], rtol=1e-13, atol=1e-9)
    assert e1.argmax == e0.argmax and e1.n_above == e0.n_above


@pytest.mark.parametrize("q", [(3, 1), (2, 2), (4, 0), (0, 4)])
def test_cross_correlation_at_the_true_lag(q):
    fac, alpha, spec = _centred(q)
    dl, dm = oracle.offset_grid(5, STEP)
    L = oracle.loglike_alpha_offsets(fac, [E_TRUE[0]], [E_TRUE[1]], alpha, dl, dm)[0]
    # closed form at the true lag: D = S' Mm, so ln L = S'^2 Mm / 2 - ln(Mm) / 2,
    # with Mm from the Eq. 1 profile at the cell centres
    f = disk_profile(fac.uc, fac.vc, alpha, *E_TRUE)
    mm = np.sum(fac.wsum * f * f)
    s = spec * FLUX
    qi = q[0] * 5 + q[1]
    assert L[qi] == pytest.approx(s * s * mm / 2.0 - 0.5 * np.log(mm), rel=1e-9)
    assert int(np.argmax(L)) == qi
    # the mirrored lag (a sign error of the shift) is far below
    mirror = (4 - q[0]) * 5 + (4 - q[1])
    if mirror != qi:
        assert L[qi] - L[mirror] > 1.0


def test_marginalised_fit_of_a_displaced_source_is_the_undisplaced_fit():
    p = oracle.Params()
    centre, _, _ = _centred((2, 2))
    inner, _, _ = _centred((3, 1))
    outer, _, _ = _centred((4, 0))
    _, ref = oracle.fit_source_pos(centre, FLUX, 5, STEP, p)
    _, got = oracle.fit_source_pos(inner, FLUX, 5, STEP, p)
    assert abs(got.e1 - ref.e1) < 1e-4 and abs(got.e2 - ref.e2) < 1e-4
    assert got.argmax == ref.argmax
    # the position-fixed fit of the displaced source is visibly off, the
    # marginalised one is not
    _, fixed = oracle.fit_source(outer, FLUX, p)
    _, marg = oracle.fit_source_pos(outer, FLUX, 5, STEP, p)
    assert np.hypot(fixed.e1 - ref.e1, fixed.e2 - ref.e2) > 0.05
    assert np.hypot(marg.e1 - ref.e1, marg.e2 - ref.e2) < 1e-3


def test_refinement_uses_the_marginalised_likelihood():
    p = oracle.Params()
    fac, _, _ = _centred((3, 1), wscale=1e10)     # a posterior narrower than 30 grid points
    surf, est = oracle.fit_source_pos(fac, FLUX, 5, STEP, p)
    assert est.n_above < 30
    ref = oracle.refine_source(fac, FLUX, surf, est, p, position=(5, STEP))
    fixed = oracle.refine_source(fac, FLUX, surf, est, p)
    assert ref.flags & oracle.FLAG_REFINED
    # the refined mean stays at the marginalised estimate's scale of accuracy
    assert np.hypot(ref.e1 - est.e1, ref.e2 - est.e2) < 0.02
    # and differs from refining with the position-fixed likelihood
    assert (ref.e1, ref.e2) != (fixed.e1, fixed.e2)


def test_prior_normalisation_on_a_facet_without_signal():
    """With Vbar = 0 every offset gives D = 0, so the mean over the offsets
    (the uniform prior's normalisation) leaves the position-fixed likelihood;
    a sum instead of a mean would add ln(n_side^2)."""
    fac, _, _ = _centred((2, 2))
    fac.vbar = np.zeros_like(fac.vbar)
    p = oracle.Params()
    s0, _ = oracle.fit_source(fac, FLUX, p)
    s5, _ = oracle.fit_source_pos(fac, FLUX, 5, STEP, p)
    fin = np.isfinite(s0)
    np.testing.assert_allclose(s5[fin], s0[fin], rtol=1e-13, atol=1e-10)
