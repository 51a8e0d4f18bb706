"""GPU parity of the HIP path with the oracle, element by element, on the tiny
workload (config 0: 20 antennas, 11,400 visibilities, 10 sources) and on
small variants that exercise ragged tails, several source tiles, several
channels, flagged data and empty facets.  Every call goes through the C ABI."""
import math

import numpy as np
import pytest

import oracle
from paper_2203_14071_amd import rlf, synth
from tests import gpu_common as G

pytestmark = pytest.mark.gpu


def _field(cfg_index=0, cfg=None, n_src=None, seed_shift=0, freq=None):
    cfg = synth.CONFIGS[cfg_index] if cfg is None else cfg
    if freq is not None:
        import dataclasses
        cfg = dataclasses.replace(cfg, freq_hz=tuple(freq))
    o = synth.observation(cfg_index, cfg)
    cat = synth.catalogue(cfg, synth.rng(cfg_index, synth.STREAM_CAT + seed_shift), n_src)
    nz = synth.noise(cfg, synth.rng(cfg_index, synth.STREAM_NOISE + seed_shift), o.n_rows * o.n_chan)
    data = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat) + nz
    return cfg, o, cat, data


def _run_all(o, cat, data, ctx, p=oracle.Params(), prior_mu=None):
    """GPU: residual against the circular sky model, extraction, fit."""
    torch = G.torch_cuda()
    catc = G.circular(cat)
    obs = G.make_obs(o, data)
    resid = torch.empty_like(obs.vis)
    ctx.model_vis(obs, catc, resid, mode=rlf.RLF_MODEL_RESIDUAL)
    f = ctx.facets_create(obs, catc, prior_mu=prior_mu)
    ctx.extract_facets(obs, catc, resid, f, prior_mu=prior_mu)
    out = G.fit_out_tensors(cat.n_src)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    return resid.cpu().numpy(), f.copy(), G.host(out), f


def _oracle_all(o, cat, data, p=oracle.Params(), mu=None):
    catc = G.circular(cat)
    resid = data - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc, p.ref_freq_hz, p.beta)
    facets = [G.oracle_facet(o, resid, catc, s, p) for s in range(cat.n_src)]
    fits = [oracle.fit_source(facets[s], cat.flux_jy[s], p, None if mu is None else mu[s])
            for s in range(cat.n_src)]
    return resid, facets, fits


@pytest.fixture(scope="module")
def ctx():
    return rlf.Context(0)


def test_model_vis_matches_oracle_cfg0(ctx):
    torch = G.torch_cuda()
    cfg, o, cat, data = _field(0)
    obs = G.make_obs(o, data)
    out = torch.empty_like(obs.vis)
    ctx.model_vis(obs, cat, out, mode=rlf.RLF_MODEL_WRITE)
    ref = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat)
    ctx.sync()
    got = out.cpu().numpy()
    bound = G.VIS_RTOL_L1 * np.sum(cat.flux_jy)
    assert np.max(np.abs(got - ref)) <= bound
    # accumulate mode adds onto what is there; a sub-range of sources sums to the whole
    ctx.model_vis(obs, cat, out, mode=rlf.RLF_MODEL_WRITE, src_begin=0, src_end=4)
    ctx.model_vis(obs, cat, out, mode=rlf.RLF_MODEL_ACCUMULATE, src_begin=4, src_end=cat.n_src)
    ctx.sync()
    assert np.max(np.abs(out.cpu().numpy() - ref)) <= 2 * bound


def test_full_path_matches_oracle_cfg0(ctx):
    cfg, o, cat, data = _field(0)
    resid_g, fac_g, out_g, f = _run_all(o, cat, data, ctx)
    resid_o, fac_o, fits_o = _oracle_all(o, cat, data)
    assert np.max(np.abs(resid_g - resid_o)) <= G.VIS_RTOL_L1 * np.sum(cat.flux_jy)
    # the GPU facets come from the GPU residual, the oracle's from its own
    scale = np.max(np.abs(resid_o))
    for s in range(cat.n_src):
        G.check_facet(fac_g, s, fac_o[s], scale, cat.flux_jy[s])
    for s in range(cat.n_src):
        surf_o, est_o = fits_o[s]
        G.check_fit(out_g, s, surf_o, G.oracle_estimate_variants(surf_o), out_g["surface"][s])
    # integer invariants of the gridding
    for s in range(cat.n_src):
        a, b = fac_g["offsets"][s], fac_g["offsets"][s + 1]
        assert fac_g["count"][a:b].sum() == o.n_rows
    f.free()


def test_ragged_multichannel_many_sources(ctx):
    """3 channels, 70 sources (three source tiles, ragged), 13 antennas x 37
    samples (2,886 rows: ragged against 512-row wave chunks), flagged
    visibilities, prior medians given per source."""
    cfg = synth.small_config(0, n_ant=13, n_time=37, n_src=70)
    freq = (1.2e9, 1.4e9, 1.55e9)
    import dataclasses
    cfg = dataclasses.replace(cfg, freq_hz=freq)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(21))
    rng = np.random.default_rng(22)
    n = o.n_rows * o.n_chan
    o.weight = o.weight * rng.uniform(0.5, 1.5, n)
    o.weight[rng.random(n) < 0.07] = 0.0
    o.weight[rng.random(n) < 0.02] = -1.0
    data = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat) + \
        cfg.noise_sigma_jy * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    mu = rng.normal(0.0, 0.2, cat.n_src)
    p = oracle.Params()
    resid_g, fac_g, out_g, f = _run_all(o, cat, data, ctx, prior_mu=mu)
    resid_o, fac_o, fits_o = _oracle_all(o, cat, data, mu=mu)
    scale = np.max(np.abs(resid_o))
    assert np.max(np.abs(resid_g - resid_o)) <= G.VIS_RTOL_L1 * np.sum(cat.flux_jy) * 2 ** 0.7
    for s in range(cat.n_src):
        G.check_facet(fac_g, s, fac_o[s], scale, cat.flux_jy[s] * 1.2)
        a, b = fac_g["offsets"][s], fac_g["offsets"][s + 1]
        assert fac_g["count"][a:b].sum() == np.count_nonzero(o.weight > 0)
    for s in range(0, cat.n_src, 7):
        surf_o, est_o = fits_o[s]
        G.check_fit(out_g, s, surf_o, G.oracle_estimate_variants(surf_o), out_g["surface"][s])
    f.free()


def test_all_flagged_gives_empty_facets(ctx):
    torch = G.torch_cuda()
    cfg, o, cat, data = _field(0)
    o.weight = np.zeros_like(o.weight)
    obs = G.make_obs(o, data)
    f = ctx.facets_create(obs, cat)
    ctx.extract_facets(obs, cat, obs.vis, f)
    out = G.fit_out_tensors(cat.n_src)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    h = G.host(out)
    n_src, n_cells, _ = f.info()
    assert n_cells == 0
    assert np.all(h["flags"] == rlf.RLF_FLAG_EMPTY)
    assert np.all(np.isnan(h["e1"])) and np.all(h["argmax"] == -1) and np.all(h["n_above"] == 0)
    assert np.all(np.isneginf(h["surface"]))
    f.free()


@pytest.mark.parametrize("fused", [False, True])
def test_single_visibility_single_source(ctx, fused):
    """Smallest input: one row, one channel, one source (one extraction wave
    and seven empty blocks of the XCD-rounded grid), through the explicit and
    the library-computed residual: one cell, and the fit of that cell."""
    g = np.random.default_rng(77)
    o = synth.observation(0)
    row = 1234
    o1 = synth.Observation(o.u_m[row:row + 1].copy(), o.v_m[row:row + 1].copy(), o.w_m[row:row + 1].copy(),
                           o.freq_hz.copy(), np.array([2.5e7]))
    cat = synth.Catalogue(np.array([0.002]), np.array([-0.001]), np.array([80e-6]), np.array([1.2]),
                          np.array([0.2]), np.array([-0.1]))
    data = oracle.sky_model(o1.u_m, o1.v_m, o1.w_m, o1.freq_hz, cat) + (1e-5 + 2e-5j) * g.standard_normal(1)
    catc = G.circular(cat)
    obs = G.make_obs(o1, data)
    f = ctx.facets_create(obs, catc)
    if fused:
        ctx.extract_facets(obs, catc, None, f)
    else:
        torch = G.torch_cuda()
        res = torch.empty_like(obs.vis)
        ctx.model_vis(obs, catc, res, mode=rlf.RLF_MODEL_RESIDUAL)
        ctx.extract_facets(obs, catc, res, f)
    out = G.fit_out_tensors(1)
    ctx.fit_sources(f, out, want_surface=True)
    ctx.sync()
    fac, h = f.copy(), G.host(out)
    resid = data - oracle.sky_model(o1.u_m, o1.v_m, o1.w_m, o1.freq_hz, catc)
    ref = G.oracle_facet(o1, resid, catc, 0)
    assert ref.n_cells == 1
    G.check_facet(fac, 0, ref, float(np.max(np.abs(resid))), cat.flux_jy[0])
    surf, _ = oracle.fit_source(ref, cat.flux_jy[0])
    G.check_fit(h, 0, surf, G.oracle_estimate_variants(surf), h["surface"][0])
    f.free()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_small_catalogue_extraction_kernel(precision):
    """Catalogues of at most eight sources go through the visibility-parallel
    extraction kernel: the same facets (cells bit-exact, sums to rounding) as
    the source-parallel kernel gives for those sources inside a nine-source
    catalogue, with the residual handed over explicitly."""
    mixed = precision == "mixed"
    c = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED if mixed else rlf.RLF_FP64))
    cfg = synth.small_config(0, n_ant=20, n_time=40, n_src=9)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(5))
    rng = np.random.default_rng(6)
    n = o.n_rows * o.n_chan
    resid = cfg.noise_sigma_jy * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    o.weight[::17] = 0.0                                           # some flagged rows
    obs = G.make_obs(o, resid.astype(np.complex64) if mixed else resid, mixed=mixed)
    res = {}
    for k in (8, 9):
        sub = cat.subset(np.arange(k))
        f = c.facets_create(obs, sub)
        c.extract_facets(obs, sub, obs.vis, f)
        res[k] = f.copy()
        f.free()
    a, b = res[8], res[9]
    for s in range(8):
        x0, x1 = a["offsets"][s], a["offsets"][s + 1]
        y0, y1 = b["offsets"][s], b["offsets"][s + 1]
        for key in ("ix", "iy", "count"):
            assert np.array_equal(a[key][x0:x1], b[key][y0:y1]), (s, key)
        assert np.allclose(a["wsum"][x0:x1], b["wsum"][y0:y1], rtol=1e-13)
        scale = np.max(np.abs(resid)) + cat.flux_jy[s]
        assert np.max(np.abs(a["vbar"][x0:x1] - b["vbar"][y0:y1])) <= (1e-5 if mixed else 1e-12) * scale
    c.close()


def test_repeat_extraction_is_self_cleaning(ctx):
    """A second extraction on the same facet object gives the same cells
    (the compaction step clears the accumulators)."""
    torch = G.torch_cuda()
    cfg, o, cat, data = _field(0)
    obs = G.make_obs(o, data)
    f = ctx.facets_create(obs, cat)
    ctx.extract_facets(obs, cat, obs.vis, f)
    a = f.copy()
    ctx.extract_facets(obs, cat, obs.vis, f)
    b = f.copy()
    for k in ("offsets", "ix", "iy", "count"):
        assert np.array_equal(a[k], b[k])
    assert np.allclose(a["vbar"], b["vbar"], rtol=1e-12, atol=1e-18)
    f.free()


def test_abi_errors_on_gpu(ctx):
    torch = G.torch_cuda()
    cfg, o, cat, data = _field(0)
    obs = G.make_obs(o, data)
    bad = cat.with_shape(np.full(cat.n_src, 0.9), np.full(cat.n_src, 0.5))      # |e| >= 1
    with pytest.raises(rlf.RlfError) as e:
        ctx.model_vis(obs, bad, torch.empty_like(obs.vis))
    assert e.value.code == rlf.RLF_EINVAL
    f = ctx.facets_create(obs, cat)
    other = synth.Catalogue(cat.l, cat.m, cat.flux_jy, cat.alpha_arcsec * 1.01, cat.e1, cat.e2)
    with pytest.raises(rlf.RlfError) as e:
        ctx.extract_facets(obs, other, obs.vis, f)
    assert e.value.code == rlf.RLF_EINVAL
    big = synth.Catalogue(cat.l, cat.m, cat.flux_jy, np.full(cat.n_src, 3e4), cat.e1, cat.e2)
    with pytest.raises(rlf.RlfError) as e:
        ctx.facets_create(obs, big)
    assert e.value.code == rlf.RLF_ERANGE
    with pytest.raises(rlf.RlfError) as e:
        ctx.model_vis(obs, cat, torch.empty_like(obs.vis), src_begin=3, src_end=99)
    assert e.value.code == rlf.RLF_EINVAL
    f.free()


def test_fused_residual_matches_explicit_residual(ctx):
    """rlf_extract_facets with residual = NULL (the library subtracts the sky
    model itself, in its sorted order) equals extraction from the residual of
    rlf_model_vis, and the oracle; 2 channels, flagged data."""
    import dataclasses
    torch = G.torch_cuda()
    cfg = dataclasses.replace(synth.small_config(0, n_ant=11, n_time=31, n_src=23), freq_hz=(1.3e9, 1.45e9))
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(41))
    rng = np.random.default_rng(42)
    n = o.n_rows * o.n_chan
    o.weight[rng.random(n) < 0.05] = 0.0
    data = oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, cat) + \
        cfg.noise_sigma_jy * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    catc = G.circular(cat)
    obs = G.make_obs(o, data)
    resid = torch.empty_like(obs.vis)
    ctx.model_vis(obs, catc, resid, mode=rlf.RLF_MODEL_RESIDUAL)
    f1 = ctx.facets_create(obs, catc)
    ctx.extract_facets(obs, catc, resid, f1)
    a = f1.copy()
    ctx.extract_facets(obs, catc, None, f1)
    b = f1.copy()
    for k in ("offsets", "ix", "iy", "count"):
        assert np.array_equal(a[k], b[k]), k
    resid_o = data - oracle.sky_model(o.u_m, o.v_m, o.w_m, o.freq_hz, catc)
    scale = np.max(np.abs(resid_o))
    for s in range(cat.n_src):
        ref = G.oracle_facet(o, resid_o, catc, s)
        G.check_facet(a, s, ref, scale, cat.flux_jy[s] * 1.1)
        G.check_facet(b, s, ref, scale, cat.flux_jy[s] * 1.1)
    f1.free()


@pytest.mark.parametrize("K", [20.0, 100.0])
def test_facet_size_factor_matches_oracle(K):
    """The facet-size factor K (Sec. 2.3) at the ends of the tuning scan."""
    import dataclasses
    cfg, o, cat, data = _field(0)
    p = dataclasses.replace(oracle.Params(), K=K)
    kctx = rlf.Context(0, None, rlf.params(K=K))
    resid_g, fac_g, out_g, f = _run_all(o, cat, data, kctx)
    resid_o, fac_o, fits_o = _oracle_all(o, cat, data, p)
    scale = np.max(np.abs(resid_o))
    for s in range(cat.n_src):
        G.check_facet(fac_g, s, fac_o[s], scale, cat.flux_jy[s])
        surf_o, est_o = fits_o[s]
        G.check_fit(out_g, s, surf_o, G.oracle_estimate_variants(surf_o, p), out_g["surface"][s])
    f.free()
    kctx.close()


def _morton_changes(u, v, theta):
    """Cell changes along a Z-order of the points (the test's own ordering, a
    check that the input really alternates between cells)."""
    def spread(x):
        x = x & 0xffff
        x = (x | (x << 8)) & 0x00ff00ff
        x = (x | (x << 4)) & 0x0f0f0f0f
        x = (x | (x << 2)) & 0x33333333
        return (x | (x << 1)) & 0x55555555
    q = lambda t: np.clip(np.floor((t / (2 * np.abs(t).max()) + 0.5) * 65536), 0, 65535).astype(np.int64)
    order = np.argsort(spread(q(u)) | (spread(q(v)) << 1), kind="stable")
    key = np.rint(v[order] * theta) * 1e6 + np.rint(u[order] * theta)
    return int(np.count_nonzero(key[1:] != key[:-1])), int(np.unique(key).size)


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
@pytest.mark.parametrize("n_src", [150, 5])
def test_boundary_crossing_runs(precision, n_src):
    """Visibilities packed densely around cell boundaries, so that along the
    sorted order every source moves back and forth between neighbouring cells
    many times: 150 sources (three source tiles of the source-parallel
    kernel: open runs swapped, older runs flushed on a third cell) and 5
    sources (the visibility-parallel kernel: short runs inside and across
    the lanes of a step), cells and counts bit-exact against the oracle,
    sums to rounding."""
    mixed = precision == "mixed"
    c = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED if mixed else rlf.RLF_FP64))
    g = np.random.default_rng(2024)
    alpha = np.exp(g.normal(0.0, 0.3, n_src))
    cat = synth.Catalogue(g.uniform(-2e-3, 2e-3, n_src), g.uniform(-2e-3, 2e-3, n_src),
                          g.uniform(20e-6, 200e-6, n_src), alpha,
                          g.uniform(-0.5, 0.5, n_src), g.uniform(-0.5, 0.5, n_src))
    cell = 1.0 / np.median(oracle.facet_theta(alpha))               # median cell side in wavelengths
    centres = g.uniform(-20 * cell, 20 * cell, (12, 2))
    u = np.concatenate([cu + g.uniform(-cell, cell, 1500) for cu, _ in centres])
    v = np.concatenate([cv + g.uniform(-cell, cell, 1500) for _, cv in centres])
    n = u.size
    w = g.uniform(-50.0, 50.0, n)
    wt = g.uniform(0.5, 2.0, n)
    wt[g.random(n) < 0.05] = 0.0                                     # flagged
    resid = 1e-4 * (g.standard_normal(n) + 1j * g.standard_normal(n))
    if mixed:
        resid = resid.astype(np.complex64).astype(np.complex128)
        wt = wt.astype(np.float32).astype(np.float64)
    freq = np.array([synth.C_LIGHT])                                 # metres = wavelengths
    changes, cells = _morton_changes(u, v, oracle.facet_theta(np.median(alpha)))
    assert changes > 8 * cells                                        # the input does alternate
    obs = rlf.Obs(G.to_dev(u), G.to_dev(v), G.to_dev(w), freq, G.complex_to_dev(resid, mixed),
                  G.to_dev(wt.astype(np.float32) if mixed else wt))
    f = c.facets_create(obs, cat)
    c.extract_facets(obs, cat, obs.vis, f)
    fac = f.copy()
    scale = float(np.max(np.abs(resid)))
    for s in range(n_src):
        theta = oracle.facet_theta(cat.alpha_arcsec[s])
        src = (cat.l[s], cat.m[s], cat.flux_jy[s], cat.alpha_arcsec[s], cat.e1[s], cat.e2[s])
        ref = oracle.extract_facet(u, v, w, freq, wt, resid, src, theta)
        if not mixed:
            G.check_facet(fac, s, ref, scale, cat.flux_jy[s])
            continue
        a, b = int(fac["offsets"][s]), int(fac["offsets"][s + 1])
        assert b - a == ref.n_cells, s
        for key in ("ix", "iy", "count"):
            assert np.array_equal(fac[key][a:b], getattr(ref, key)), (s, key)
        assert np.allclose(fac["wsum"][a:b], ref.wsum, rtol=1e-12), s
        assert np.max(np.abs(fac["vbar"][a:b] - ref.vbar)) <= 2e-5 * (scale + cat.flux_jy[s]), s
    f.free()
    c.close()


@pytest.mark.parametrize("precision", ["fp64", "mixed"])
def test_zero_flux_sources(precision):
    """Sources of zero flux (some circular) in a catalogue of 12 (the
    source-parallel kernel): their own model is zero, so their facets are the
    shifted residual alone, against the oracle; a negative flux is rejected."""
    mixed = precision == "mixed"
    c = rlf.Context(0, None, rlf.params(precision=rlf.RLF_MIXED if mixed else rlf.RLF_FP64))
    cfg = synth.small_config(0, n_ant=16, n_time=30, n_src=12)
    o = synth.observation(0, cfg)
    cat = synth.catalogue(cfg, np.random.default_rng(41))
    flux = cat.flux_jy.copy()
    flux[[1, 4, 7, 10]] = 0.0
    e1, e2 = cat.e1.copy(), cat.e2.copy()
    e1[[4, 10]] = 0.0
    e2[[4, 10]] = 0.0
    cat = synth.Catalogue(cat.l, cat.m, flux, cat.alpha_arcsec, e1, e2)
    rng = np.random.default_rng(42)
    n = o.n_rows * o.n_chan
    resid = cfg.noise_sigma_jy * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    if mixed:
        resid = resid.astype(np.complex64).astype(np.complex128)
        o.weight = o.weight.astype(np.float32).astype(np.float64)
    obs = G.make_obs(o, resid, mixed=mixed)
    mu = np.full(cat.n_src, 0.1)                                    # the Eq. 4 prior needs a positive flux
    f = c.facets_create(obs, cat, prior_mu=mu)
    c.extract_facets(obs, cat, obs.vis, f, prior_mu=mu)
    fac = f.copy()
    scale = float(np.max(np.abs(resid)))
    for s in range(cat.n_src):
        ref = G.oracle_facet(o, resid, cat, s)
        a, b = int(fac["offsets"][s]), int(fac["offsets"][s + 1])
        assert b - a == ref.n_cells, s
        for key in ("ix", "iy", "count"):
            assert np.array_equal(fac[key][a:b], getattr(ref, key)), (s, key)
        tol = (2e-5 if mixed else G.VBAR_TOL) * (scale + cat.flux_jy[s])
        assert np.all(np.isfinite(fac["vbar"][a:b])), s
        assert np.max(np.abs(fac["vbar"][a:b] - ref.vbar)) <= tol, s
    f.free()
    bad = synth.Catalogue(cat.l, cat.m, np.where(np.arange(cat.n_src) == 3, -1e-5, flux), cat.alpha_arcsec, e1, e2)
    with pytest.raises(rlf.RlfError) as e:
        c.facets_create(obs, bad, prior_mu=mu)
    assert e.value.code == rlf.RLF_EINVAL
    c.close()


def test_extraction_table_sizes_agree():
    """The FP64 extraction takes a 2048-entry exp table for launches of at
    least 8 source tiles (512 sources) and a 1024-entry one below: 600
    sources extracted together (10 tiles) and the same sources in two
    halves (5 tiles each) give the same cells, counts and weight sums
    (weight sums to their summation order, exact or within a few ulp) and
    facet averages within the two tables' difference (each within 2.3e-16
    of exp(2 pi i phi) per term)."""
    cfg = synth.CONFIGS[0]
    o = synth.observation(0, cfg)
    cat = G.circular(synth.catalogue(cfg, synth.rng(0, synth.STREAM_CAT + 11), 600))
    rng = np.random.default_rng(11)
    n = o.n_rows * o.n_chan
    resid = cfg.noise_sigma_jy * (rng.standard_normal(n) + 1j * rng.standard_normal(n))
    c = rlf.Context(0)
    obs = G.make_obs(o, resid)

    def extract(sub):
        f = c.facets_create(obs, sub)
        c.extract_facets(obs, sub, obs.vis, f)
        fac = f.copy()
        f.free()
        return fac

    full = extract(cat)
    halves = [extract(cat.subset(np.arange(0, 300))), extract(cat.subset(np.arange(300, 600)))]
    scale = float(np.max(np.abs(resid)))
    for s in range(cat.n_src):
        h, t = halves[s // 300], s % 300
        a, b = int(full["offsets"][s]), int(full["offsets"][s + 1])
        ha, hb = int(h["offsets"][t]), int(h["offsets"][t + 1])
        assert b - a == hb - ha > 0, s
        for key in ("ix", "iy", "count"):
            assert np.array_equal(full[key][a:b], h[key][ha:hb]), (s, key)
        assert np.allclose(full["wsum"][a:b], h["wsum"][ha:hb], rtol=1e-13, atol=0), s
        tol = 1e-14 * (scale + cat.flux_jy[s])
        assert np.max(np.abs(full["vbar"][a:b] - h["vbar"][ha:hb])) <= tol, s
    c.close()
