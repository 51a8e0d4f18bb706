"""Position marginalisation (rlf_facets_set_positions) against the oracle's
fit_source_pos: full-grid surfaces and estimates in the FP64 form for 3x3,
5x5 and 7x7 offset grids and in the mixed form, a noiseless source displaced
from its catalogue position by a grid offset, the adaptive refinement on the
marginalised likelihood, and the argument errors."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle.model import ARCSEC, C_LIGHT
from oracle.position import fit_source_pos
from oracle.refine import FLAG_REFINED, refine_source
from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _field(seed, n_src=4, noise_scale=1.0):
    cfg = synth.small_config(0, n_ant=12, n_time=20, n_src=n_src)
    cfg = dataclasses.replace(cfg, noise_sigma_jy=noise_scale * cfg.noise_sigma_jy)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(seed))
    rng = np.random.default_rng(seed + 1)
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    vis = vis + cfg.noise_sigma_jy * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))
    return o, cat, vis


def _gpu_fit(ctx, o, vis, catc, n_side, step, mixed=False, refine=False):
    obs = G.make_obs(o, vis.astype(np.complex64) if mixed else vis, mixed=mixed)
    f = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, None, f)
    ctx.set_positions(f, n_side, step)
    out = G.fit_out_tensors(catc.n_src)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    coarse = G.host(out)
    h = None
    if refine:
        ctx.refine_sources(f, out)
        ctx.sync()
        h = G.host(out)
    f.free()
    return coarse, h


@pytest.mark.parametrize("n_side,step", [(3, 0.2), (5, 0.15), (7, 0.1)])
def test_fp64_against_oracle(n_side, step):
    o, cat, vis = _field(11)
    catc = G.circular(cat)
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc)
    ctx = rlf.Context(0)
    h, _ = _gpu_fit(ctx, o, vis, catc, n_side, step)
    for s in range(cat.n_src):
        fac = G.oracle_facet(o, resid, catc, s)
        surf, _ = fit_source_pos(fac, cat.flux_jy[s], n_side, step)
        G.check_fit(h, s, surf, G.oracle_estimate_variants(surf), h["surface"][s])
    ctx.close()


def test_mixed_against_oracle():
    o, cat, vis = _field(12)
    o.weight = o.weight.astype(np.float32).astype(np.float64)
    vis = vis.astype(np.complex64).astype(np.complex128)      # the inputs the mixed form sees
    catc = G.circular(cat)
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc)
    ctx = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED))
    h, _ = _gpu_fit(ctx, o, vis, catc, 5, 0.15, mixed=True)
    worst = 0.0
    for s in range(cat.n_src):
        fac = G.oracle_facet(o, resid, catc, s)
        surf, est = fit_source_pos(fac, cat.flux_jy[s], 5, 0.15)
        fin = np.isfinite(surf)
        assert np.array_equal(fin, np.isfinite(h["surface"][s]))
        # FP32 profile and cross-correlation sums: ln L within 1e-4 relative
        d = np.abs(h["surface"][s][fin] - surf[fin])
        assert np.all(d <= 1e-4 * np.maximum(1.0, np.abs(surf[fin]))), (s, d.max())
        assert abs(h["e1"][s] - est.e1) <= 1e-4 and abs(h["e2"][s] - est.e2) <= 1e-4, s
        worst = max(worst, float(d.max()))
    print(f"mixed position marginalisation: max |dl| {worst:.2e}")
    ctx.close()


def _displaced(q, step=0.3, n_side=5, seed=3):
    """A noiseless source displaced by offset q of the grid from its catalogue
    position; one channel at nu = c, w = 0, visibilities at cell centres."""
    rng = np.random.default_rng(seed)
    alpha = oracle.alpha_knots()[10]
    theta = oracle.facet_theta(alpha)
    g = np.arange(-14, 15)
    IX, IY = np.meshgrid(g, g, indexing="ij")
    keep = rng.random(IX.size) < 0.6
    u, v = IX.reshape(-1)[keep] / theta, IY.reshape(-1)[keep] / theta
    n = u.shape[0]
    h = (n_side - 1) // 2
    l0, m0 = 0.001, -0.0005
    truth = synth.Catalogue(np.array([l0 + (q[0] - h) * step * ARCSEC]), np.array([m0 + (q[1] - h) * step * ARCSEC]),
                            np.array([100e-6]), np.array([alpha]), np.array([0.3]), np.array([-0.2]))
    cat = synth.Catalogue(np.array([l0]), np.array([m0]), np.array([100e-6]), np.array([alpha]),
                          np.array([0.3]), np.array([-0.2]))
    freq = np.array([C_LIGHT])
    vis = oracle.sky_model(u, v, np.zeros(n), freq, truth)
    w = rng.uniform(0.5, 2.0, n) * 1e8
    return u, v, freq, w, vis, cat


def test_displaced_source_on_cell_centres():
    ctx = rlf.Context(0)
    ests = {}
    for q in ((2, 2), (3, 1)):
        u, v, freq, w, vis, cat = _displaced(q)
        n = u.shape[0]
        obs = rlf.Obs(G.to_dev(u), G.to_dev(v), G.to_dev(np.zeros(n)), freq, G.complex_to_dev(vis), G.to_dev(w))
        f = ctx.facets_create(obs, cat)
        ctx.extract_facets(obs, cat, None, f)
        ctx.set_positions(f, 5, 0.3)
        out = G.fit_out_tensors(1)
        ctx.fit_sources(f, out, want_surface=True)
        ctx.sync()
        h = G.host(out)
        resid = vis - oracle.sky_model(u, v, np.zeros(n), freq, cat)
        fac = oracle.extract_facet(u, v, np.zeros(n), freq, w, resid,
                                   (cat.l[0], cat.m[0], cat.flux_jy[0], cat.alpha_arcsec[0], cat.e1[0], cat.e2[0]),
                                   oracle.facet_theta(cat.alpha_arcsec[0]))
        surf, _ = fit_source_pos(fac, cat.flux_jy[0], 5, 0.3)
        G.check_fit(h, 0, surf, G.oracle_estimate_variants(surf), h["surface"][0])
        ests[q] = (h["e1"][0], h["e2"][0])
        f.free()
    # displaced by an interior offset: the marginalised estimate is the undisplaced one
    assert abs(ests[(3, 1)][0] - ests[(2, 2)][0]) < 1e-4 and abs(ests[(3, 1)][1] - ests[(2, 2)][1]) < 1e-4
    ctx.close()


def _robust_refine(fac, flux, surf, est, p, position):
    d = 16 * G.LL_RTOL * max(1.0, abs(est.lmax))
    runs = [refine_source(fac, flux, surf, est, dataclasses.replace(p, frac=p.frac * math.exp(x)), position=position)
            for x in (0.0, -d, d)]
    for r in runs[1:]:
        if r.n_above != runs[0].n_above or r.flags != runs[0].flags or abs(r.e1 - runs[0].e1) > 1e-12:
            return None
    return runs[0]


def test_refinement_with_positions_against_oracle():
    o, cat, vis = _field(21, n_src=8, noise_scale=0.05)
    catc = G.circular(cat)
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc)
    p = oracle.Params()
    ctx = rlf.Context(0)
    coarse, h = _gpu_fit(ctx, o, vis, catc, 3, 0.1, refine=True)
    checked = refined = 0
    for s in range(cat.n_src):
        fac = G.oracle_facet(o, resid, catc, s)
        surf, est = fit_source_pos(fac, cat.flux_jy[s], 3, 0.1, p)
        ref = _robust_refine(fac, cat.flux_jy[s], surf, est, p, (3, 0.1))
        if ref is None or int(coarse["n_above"][s]) != est.n_above:
            continue
        checked += 1
        refined += bool(ref.flags & FLAG_REFINED)
        assert int(h["flags"][s]) == ref.flags, s
        assert int(h["n_above"][s]) == ref.n_above, s
        for k in ("e1", "e2", "s1", "s2", "c12"):
            assert abs(h[k][s] - getattr(ref, k)) <= G.E_TOL, (s, k)
        assert abs(h["lmax"][s] - ref.lmax) <= G.LL_RTOL * max(1.0, abs(ref.lmax))
    print(f"refinement with positions: {checked} checked, {refined} refined")
    assert checked >= 6 and refined >= 3
    ctx.close()


def test_position_argument_errors_and_reset():
    o, cat, vis = _field(31, n_src=3)
    catc = G.circular(cat)
    ctx = rlf.Context(0)
    obs = G.make_obs(o, vis)
    f = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, None, f)
    for n_side, step in ((2, 0.1), (9, 0.1), (0, 0.1), (3, 0.0), (3, -1.0), (3, float("nan"))):
        with pytest.raises(rlf.RlfError) as e:
            ctx.set_positions(f, n_side, step)
        assert e.value.code == rlf.RLF_EINVAL
    plain = G.fit_out_tensors(3)
    ctx.fit_sources(f, plain, want_surface=True)
    ctx.set_positions(f, 3, 0.2)
    win = G.to_dev(np.tile(np.array([30, 50, 30, 50], np.int32), 3))
    with pytest.raises(rlf.RlfError) as e:
        ctx.fit_sources(f, G.fit_out_tensors(3), mode=1, window=win)
    assert e.value.code == rlf.RLF_EUNSUPPORTED
    with pytest.raises(rlf.RlfError) as e:
        ctx.fit_sources(f, G.fit_out_tensors(3), mode=2, check_stride=4)
    assert e.value.code == rlf.RLF_EUNSUPPORTED
    # back to the fixed position: the same kernel as a facet object never set
    ctx.set_positions(f, 1)
    again = G.fit_out_tensors(3)
    ctx.fit_sources(f, again, want_surface=True)
    ctx.sync()
    a, b = G.host(plain), G.host(again)
    assert np.array_equal(a["surface"], b["surface"])
    f.free()
    ctx.close()
