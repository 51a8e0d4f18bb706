"""Pins of the sequential sky-model refinement oracle (Sec. 2.1, 2.4, 3.1):
its one-chunk case is the data-parallel pass, serial refinement cleans a
faint source's facet of a bright neighbour's shape, and the bad-fit refit
bookkeeping follows its definition."""
import dataclasses

import numpy as np
import pytest

import oracle
from oracle.estimate import FLAG_BAD_VAR, FLAG_EMPTY
from oracle.sequential import FLAG_REFIT, SkyCatalogue, fit_sequential
from paper_2203_14071_amd import synth


def _field(n_src=3, seed=5, noise=True):
    cfg = synth.small_config(0, n_ant=12, n_time=20, n_src=n_src)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(seed))
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    if noise:
        rng = np.random.default_rng(seed + 1)
        vis = vis + cfg.noise_sigma_jy * (rng.standard_normal(vis.size) + 1j * rng.standard_normal(vis.size))
    start = SkyCatalogue(cat.l, cat.m, cat.flux_jy, cat.alpha_arcsec, np.zeros(n_src), np.zeros(n_src))
    return o, vis, cat, start


def test_one_chunk_is_the_data_parallel_pass():
    o, vis, cat, start = _field()
    p = oracle.Params()
    est, e1, e2 = fit_sequential(o, vis, start, chunk=len(cat.l), refit_bad=False, p=p)
    resid = vis - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, start)
    for s in range(len(cat.l)):
        src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], 0.0, 0.0)
        fac = oracle.extract_facet(o.u_m, o.v_m, o.w_m, o.freq_hz, o.weight, resid, src,
                                   oracle.facet_theta(cat.alpha_arcsec[s]))
        ref = oracle.fit_source(fac, cat.flux_jy[s], p)[1]
        assert dataclasses.astuple(est[s]) == dataclasses.astuple(ref)
        good = not ref.flags & (FLAG_BAD_VAR | FLAG_EMPTY)
        assert (e1[s], e2[s]) == ((ref.e1, ref.e2) if good else (0.0, 0.0))


def test_serial_refinement_removes_a_bright_neighbours_shape():
    """Noiseless pair 8 arcsec apart: a bright elongated source A and a
    fainter round source B.  Fitted together from circular models, B's facet
    holds A's shape residual; fitted after A (chunk 1), A's measured shape is
    in the model and B's estimate moves to within half the distance of B's
    estimate in isolation."""
    cfg = synth.small_config(0, n_ant=12, n_time=20, n_src=2)
    o = synth.observation(0, cfg)
    sep = 8.0 * oracle.ARCSEC
    cat = SkyCatalogue(np.array([0.001, 0.001 + sep]), np.array([-0.0005, -0.0005]),
                       np.array([200e-6, 50e-6]), np.array([1.5, 1.0]),
                       np.array([0.6, 0.0]), np.array([0.2, 0.0]))
    vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    start = dataclasses.replace(cat, e1=np.zeros(2), e2=np.zeros(2))
    p = dataclasses.replace(oracle.Params(), bad_sigma=0.0, bad_sqrtdet=0.0)
    serial, _, _ = fit_sequential(o, vis, start, chunk=1, refit_bad=False, p=p)
    joint, _, _ = fit_sequential(o, vis, start, chunk=2, refit_bad=False, p=p)
    only_b = SkyCatalogue(*(np.array([getattr(start, k)[1]]) for k in
                            ("l", "m", "flux_jy", "alpha_arcsec", "e1", "e2")))
    alone_vis = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat, sources=[1])
    alone, _, _ = fit_sequential(o, alone_vis, only_b, chunk=1, refit_bad=False, p=p)
    # A is fitted from the same data either way
    assert serial[0].e1 == joint[0].e1 and serial[0].e2 == joint[0].e2
    d_serial = np.hypot(serial[1].e1 - alone[0].e1, serial[1].e2 - alone[0].e2)
    d_joint = np.hypot(joint[1].e1 - alone[0].e1, joint[1].e2 - alone[0].e2)
    assert d_joint > 0.05 and d_serial < 0.5 * d_joint, (d_serial, d_joint)


@pytest.mark.parametrize("refit", [False, True])
def test_bad_fits_keep_their_model_and_are_refitted(refit):
    o, vis, cat, start = _field(n_src=3, seed=9)
    # a bad-variance threshold above every posterior width flags every fit
    p = dataclasses.replace(oracle.Params(), bad_sigma=10.0)
    est, e1, e2 = fit_sequential(o, vis, start, chunk=1, refit_bad=refit, p=p)
    for s in range(3):
        assert est[s].flags & FLAG_BAD_VAR
        assert bool(est[s].flags & FLAG_REFIT) == refit
    if not refit:
        assert np.all(e1 == 0.0) and np.all(e2 == 0.0)
    else:
        # no model was ever refined, so each refit sees the first residual
        first, _, _ = fit_sequential(o, vis, start, chunk=3, refit_bad=False, p=p)
        for s in range(3):
            assert est[s].e1 == first[s].e1 and est[s].e2 == first[s].e2
            assert (e1[s], e2[s]) == (est[s].e1, est[s].e2)
