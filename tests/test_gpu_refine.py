"""Adaptive refinement (rlf_refine_sources) against the oracle's
refine_source: an off-grid noiseless peak resolved to the injected shape,
and a high signal-to-noise field where most sources refine through one to
three levels."""
import dataclasses
import math

import numpy as np
import pytest

import oracle
from oracle.refine import FLAG_REFINED, refine_source
from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu

KEYS = ("e1", "e2", "s1", "s2", "c12", "lmax", "n_above", "flags")


def test_off_grid_peak_on_cell_centres():
    torch = G.torch_cuda()
    p = oracle.Params(num_r=8)
    alpha = oracle.alpha_knots(p.rmin, p.rmax, p.num_r)[4]
    theta = oracle.facet_theta(alpha)
    g = np.arange(-14, 15)
    IX, IY = np.meshgrid(g, g, indexing="ij")
    u, v = IX.reshape(-1) / theta, IY.reshape(-1) / theta
    e1, e2 = 123 * (0.02 / 8), -45 * (0.02 / 8)
    data = 2e-4 * oracle.model.disk_profile(u, v, alpha, e1, e2) + 0j
    n = u.shape[0]
    freq = np.array([299792458.0])                      # wavelengths = metres
    w = np.full(n, 1e14)
    fac = oracle.extract_facet(u, v, np.zeros(n), freq, w, data, (0.0, 0.0, 0.0, alpha, 0.0, 0.0), theta)
    surf, est = oracle.fit_source(fac, 2e-4, p, mu=math.log(alpha))
    ref = refine_source(fac, 2e-4, surf, est, p, mu=math.log(alpha))
    assert ref.e1 == pytest.approx(e1, abs=1e-9)

    ctx = rlf.Context(0, None, rlf.params(num_r=8))
    obs = rlf.Obs(G.to_dev(u), G.to_dev(v), G.to_dev(np.zeros(n)), freq, G.complex_to_dev(data), G.to_dev(w))
    cat = synth.Catalogue(np.zeros(1), np.zeros(1), np.zeros(1), np.array([alpha]), np.zeros(1), np.zeros(1))
    mu = np.array([math.log(alpha)])
    f = ctx.facets_create(obs, cat, prior_mu=mu)
    ctx.extract_facets(obs, cat, obs.vis, f, prior_mu=mu)        # zero flux: the facet is the data
    out = G.fit_out_tensors(1, surface=False)
    ctx.fit_sources(f, out)
    ctx.refine_sources(f, out, np_max=30, e_res=0.003)
    ctx.sync()
    h = G.host(out)
    assert int(h["flags"][0]) == ref.flags and ref.flags & FLAG_REFINED
    assert int(h["n_above"][0]) == ref.n_above
    for k in ("e1", "e2", "s1", "s2", "c12"):
        assert abs(h[k][0] - getattr(ref, k)) <= 1e-9, k
    assert abs(h["lmax"][0] - ref.lmax) <= 1e-9 * abs(ref.lmax)
    f.free()
    ctx.close()


def _robust(fac, flux, surf, est, p):
    """The oracle's refinement, or None when moving the threshold by a few
    LL_RTOL changes it (two correct FP64 evaluations may then differ)."""
    d = 16 * G.LL_RTOL * max(1.0, abs(est.lmax))
    runs = [refine_source(fac, flux, surf, est, dataclasses.replace(p, frac=p.frac * math.exp(x)))
            for x in (0.0, -d, d)]
    base = runs[0]
    for r in runs[1:]:
        if r.n_above != base.n_above or r.flags != base.flags or abs(r.e1 - base.e1) > 1e-12:
            return None
    return base


def test_high_snr_field_against_oracle():
    cfg = synth.small_config(0, n_ant=16, n_time=30, n_src=16)
    cfg = dataclasses.replace(cfg, noise_sigma_jy=0.05 * cfg.noise_sigma_jy)   # sharp posteriors
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(41))
    rng = np.random.default_rng(42)
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    vis = vis + cfg.noise_sigma_jy * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))
    catc = G.circular(cat)
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc)
    p = oracle.Params()
    ctx = rlf.Context(0)
    obs = G.make_obs(o, vis)
    f = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, None, f)
    out = G.fit_out_tensors(cat.n_src, surface=False)
    ctx.fit_sources(f, out)
    ctx.sync()
    coarse = G.host(out)
    ctx.refine_sources(f, out)
    ctx.sync()
    h = G.host(out)
    checked = refined = 0
    for s in range(cat.n_src):
        fac = G.oracle_facet(o, resid, catc, s)
        surf, est = oracle.fit_source(fac, cat.flux_jy[s], p)
        ref = _robust(fac, cat.flux_jy[s], surf, est, p)
        if ref is None or int(coarse["n_above"][s]) != est.n_above:
            continue
        checked += 1
        refined += bool(ref.flags & FLAG_REFINED)
        assert int(h["flags"][s]) == ref.flags, (s, int(h["flags"][s]), ref.flags)
        assert int(h["n_above"][s]) == ref.n_above, s
        for k in ("e1", "e2", "s1", "s2", "c12"):
            assert abs(h[k][s] - getattr(ref, k)) <= G.E_TOL, (s, k, h[k][s], getattr(ref, k))
        assert abs(h["lmax"][s] - ref.lmax) <= G.LL_RTOL * max(1.0, abs(ref.lmax))
    print(f"refinement: {checked} sources checked, {refined} refined")
    assert checked >= 12 and refined >= 6
    f.free()
    ctx.close()


def test_refine_argument_errors():
    cfg = synth.small_config(0, n_ant=6, n_time=5, n_src=2)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(1))
    ctx = rlf.Context(0)
    obs = G.make_obs(o, np.zeros(o.n_rows, np.complex128))
    f = ctx.facets_create(obs, cat)
    out = G.fit_out_tensors(2, surface=False)
    for kw in (dict(np_max=0), dict(e_res=0.0), dict(e_res=1e-9)):
        with pytest.raises(rlf.RlfError):
            ctx.refine_sources(f, out, **kw)
    f.free()
    ctx.close()
